// Host side of the C ABI declared in misa.h: descriptor validation, the
// lattice-id map and Neighbor Offset Index (Sec. 3), spline coefficient records
// (Sec. 4.1), placement of atoms into the Lattice List (Sec. 3, Hash
// Initialization, with the slot tolerance), and the per-step orchestration of
// the kernels on the caller's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "misa_internal.h"

using namespace misa;

// Scratch of misa_set_state_noalloc: the placement bid of every atom, then the
// counter of non-finite inputs.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code `scratch` only names the symbol: kernels
// get the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint32_t scratch[MISA_NOALLOC_MAX_ATOMS + 64];

namespace {

thread_local std::string g_create_error;

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_addr;  // per device ordinal; null until looked up

// Address of `scratch` on device dev, looked up once per device; dev must be the
// current device.
hipError_t scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

int fail(misa_lattice *h, int code, const std::string &msg) {
    if (h)
        h->err = msg;
    else
        g_create_error = msg;
    return code;
}

#define HIPCHK(h, expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((h), MISA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

int64_t next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

template <typename T>
hipError_t dev_alloc(T **p, int64_t count) {
    *p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * (size_t)count);
}

// ---------------------------------------------------------------------------
// Neighbor Offset Index: all lattice-id offsets (dX, dY, dZ) whose site lies
// strictly closer than R to a site of the given parity.

struct CanonOffset {
    int dX, dY, dZ;
    double d2;
};

std::vector<CanonOffset> enumerate_offsets(double a, double R, int parity) {
    std::vector<CanonOffset> out;
    const int w = (int)std::ceil(R / a) + 1;
    for (int dZ = -w; dZ <= w; ++dZ)
        for (int dY = -w; dY <= w; ++dY)
            for (int dX = -2 * w; dX <= 2 * w; ++dX) {
                if (!dX && !dY && !dZ) continue;
                const int pn = ((parity + dX) % 2 + 2) % 2;
                const double ox = dX * 0.5 * a;
                const double oy = (dY + 0.5 * pn - 0.5 * parity) * a;
                const double oz = (dZ + 0.5 * pn - 0.5 * parity) * a;
                const double d2 = ox * ox + oy * oy + oz * oz;
                if (d2 < R * R) out.push_back({dX, dY, dZ, d2});
            }
    // shell order (nearest first) so consecutive offsets of a wave read one band of the tables
    std::sort(out.begin(), out.end(), [](const CanonOffset &l, const CanonOffset &r) {
        if (l.d2 != r.d2) return l.d2 < r.d2;
        if (l.dZ != r.dZ) return l.dZ < r.dZ;
        if (l.dY != r.dY) return l.dY < r.dY;
        return l.dX < r.dX;
    });
    return out;
}

// ---------------------------------------------------------------------------
// spline records: local cubic Hermite per segment, node slopes from fourth-order
// central differences (second-order / one-sided next to the ends), in units of
// the sample spacing.

void node_slopes(const double *y, int n, std::vector<double> &m) {
    m.assign(n, 0.0);
    m[0] = y[1] - y[0];
    m[1] = (y[2] - y[0]) / 2.0;
    for (int k = 2; k <= n - 3; ++k) m[k] = (y[k - 2] - 8.0 * y[k - 1] + 8.0 * y[k + 1] - y[k + 2]) / 12.0;
    m[n - 2] = (y[n - 1] - y[n - 3]) / 2.0;
    m[n - 1] = y[n - 1] - y[n - 2];
}

struct SegCoef {
    double c0, c1, c2, c3;  // value in the local variable t in [0, 1]
    double d0, d1, d2;      // d/dx
};

std::vector<SegCoef> segments(const misa_table &t) {
    std::vector<double> m;
    node_slopes(t.y, t.n, m);
    std::vector<SegCoef> s(t.n - 1);
    for (int k = 0; k < t.n - 1; ++k) {
        const double dy = t.y[k + 1] - t.y[k];
        SegCoef c;
        c.c0 = t.y[k];
        c.c1 = m[k];
        c.c2 = 3.0 * dy - 2.0 * m[k] - m[k + 1];
        c.c3 = m[k] + m[k + 1] - 2.0 * dy;
        c.d0 = c.c1 / t.dx;
        c.d1 = 2.0 * c.c2 / t.dx;
        c.d2 = 3.0 * c.c3 / t.dx;
        s[k] = c;
    }
    return s;
}

template <typename Real>
TabMeta<Real> meta_of(const misa_table &t) {
    std::vector<double> m;
    node_slopes(t.y, t.n, m);
    TabMeta<Real> M{};
    M.x0 = (Real)t.x0;
    M.inv_h = (Real)(1.0 / t.dx);
    M.nseg = t.n - 1;
    M.x_last = (Real)(t.x0 + (t.n - 1) * t.dx);
    M.y_last = (Real)t.y[t.n - 1];
    M.d_last = (Real)(m[t.n - 1] / t.dx);
    return M;
}

template <typename Real>
int upload_tables(misa_lattice *h, DevTables<Real> &D, const std::vector<SegCoef> &sf,
                  const std::vector<SegCoef> &sp, const std::vector<SegCoef> &se, const misa_table &f,
                  const misa_table &e) {
    const size_t nf = sf.size(), ne = se.size();
    std::vector<Q4<Real>> F(nf), FO(2 * nf), PH(nf), EM(2 * ne);
    std::vector<Real> FO6(6 * nf);
    for (size_t k = 0; k < nf; ++k) {
        F[k] = {(Real)sf[k].c0, (Real)sf[k].c1, (Real)sf[k].c2, (Real)sf[k].c3};
        FO[2 * k] = {(Real)sf[k].d0, (Real)sf[k].d1, (Real)sf[k].d2, (Real)sp[k].d0};
        FO[2 * k + 1] = {(Real)sp[k].d1, (Real)sp[k].d2, (Real)0, (Real)0};
        const double r6[6] = {sf[k].d0, sf[k].d1, sf[k].d2, sp[k].d0, sp[k].d1, sp[k].d2};
        for (int i = 0; i < 6; ++i) FO6[6 * k + i] = (Real)r6[i];
        PH[k] = {(Real)sp[k].c0, (Real)sp[k].c1, (Real)sp[k].c2, (Real)sp[k].c3};
    }
    for (size_t k = 0; k < ne; ++k) {
        EM[2 * k] = {(Real)se[k].c0, (Real)se[k].c1, (Real)se[k].c2, (Real)se[k].c3};
        EM[2 * k + 1] = {(Real)se[k].d0, (Real)se[k].d1, (Real)se[k].d2, (Real)0};
    }
    (void)hipFree(D.f);
    (void)hipFree(D.force);
    (void)hipFree(D.phi);
    (void)hipFree(D.emb);
    (void)hipFree(D.force6);
    D.f = D.force = D.phi = D.emb = nullptr;
    D.force6 = nullptr;
    HIPCHK(h, dev_alloc(&D.f, (int64_t)nf));
    HIPCHK(h, dev_alloc(&D.force, (int64_t)(2 * nf)));
    HIPCHK(h, dev_alloc(&D.phi, (int64_t)nf));
    HIPCHK(h, dev_alloc(&D.emb, (int64_t)(2 * ne)));
    HIPCHK(h, dev_alloc(&D.force6, (int64_t)(6 * nf)));
    HIPCHK(h, hipMemcpy(D.force6, FO6.data(), sizeof(Real) * 6 * nf, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(D.f, F.data(), sizeof(Q4<Real>) * nf, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(D.force, FO.data(), sizeof(Q4<Real>) * 2 * nf, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(D.phi, PH.data(), sizeof(Q4<Real>) * nf, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(D.emb, EM.data(), sizeof(Q4<Real>) * 2 * ne, hipMemcpyHostToDevice));
    D.fm = meta_of<Real>(f);
    D.em = meta_of<Real>(e);
    return MISA_OK;
}

// ---------------------------------------------------------------------------
// state layout inside the caller's buffer

int64_t carve(misa_lattice *h, char *base, State *S, UV *alt = nullptr) {
    const int64_t ns = h->g.nsites, rc = h->rcap;
    const int64_t rs = h->precision == MISA_FP32 ? 4 : 8;
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    State s{};
    s.ux = (double *)take(8 * ns);
    s.uy = (double *)take(8 * ns);
    s.uz = (double *)take(8 * ns);
    s.vx = (double *)take(8 * ns);
    s.vy = (double *)take(8 * ns);
    s.vz = (double *)take(8 * ns);
    s.fx = take(rs * ns);
    s.fy = take(rs * ns);
    s.fz = take(rs * ns);
    s.rho = take(rs * ns);
    s.fp = take(rs * ns);
    s.atom = (int32_t *)take(4 * ns);
    s.r_id = (int32_t *)take(4 * rc);
    double **rd[] = {&s.r_x, &s.r_y, &s.r_z, &s.r_vx, &s.r_vy, &s.r_vz, &s.r_fx, &s.r_fy, &s.r_fz, &s.r_rho, &s.r_fp};
    for (double **p : rd) *p = (double *)take(8 * rc);
    s.r_e = (double *)take(16 * rc);
    UV a{};  // the second copy of u and v (the kick-drift writes one copy from the other)
    a.ux = (double *)take(8 * ns);
    a.uy = (double *)take(8 * ns);
    a.uz = (double *)take(8 * ns);
    a.vx = (double *)take(8 * ns);
    a.vy = (double *)take(8 * ns);
    a.vz = (double *)take(8 * ns);
    if (S) *S = s;
    if (alt) *alt = a;
    return off;
}

hipError_t ensure_staging(misa_lattice *h, int64_t bytes) {
    if (bytes <= h->staging_bytes) return hipSuccess;
    (void)hipFree(h->staging);
    h->staging = nullptr;
    h->staging_bytes = 0;
    hipError_t e = hipMalloc((void **)&h->staging, (size_t)bytes);
    if (e == hipSuccess) h->staging_bytes = bytes;
    return e;
}

int check_ready(misa_lattice *h, bool need_tables) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (!h->state_bound) return fail(h, MISA_ESTATE, "no state buffer bound (misa_bind_state)");
    if (!h->state_set) return fail(h, MISA_ESTATE, "no atoms loaded (misa_set_state)");
    if (need_tables && !h->tables_set) return fail(h, MISA_ESTATE, "no potential tables (misa_set_potential_tables)");
    if (need_tables && h->use_mlp && !(h->mlp.set[0] && h->mlp.set[1] && h->mlp.set[2]))
        return fail(h, MISA_ESTATE, "learned form: networks for f, phi and F not all attached (misa_set_mlp)");
    return MISA_OK;
}

hipError_t clear_marks(misa_lattice *h);

// Records HIP events around one group of launches when timing is enabled, and
// marks the group as a roctx range (rocprofv3 --marker-trace shows the phases of
// a step on the host timeline).
const char *const PHASE_NAME[MISA_TIMER_COUNT] = {"misa:rho", "misa:force", "misa:kick", "misa:runaway",
                                                  "misa:other"};
class GroupTimer {
  public:
    GroupTimer(misa_lattice *h, int cls) : h_(h), cls_(cls) {
        roctxRangePushA(PHASE_NAME[cls]);
        if (!h->timing) return;
        if (!h->event_pool.empty()) {
            ev_ = h->event_pool.back();
            h->event_pool.pop_back();
        } else if (hipEventCreate(&ev_.first) != hipSuccess || hipEventCreate(&ev_.second) != hipSuccess) {
            ev_ = {nullptr, nullptr};
            return;
        }
        if (hipEventRecord(ev_.first, h->stream) != hipSuccess) ev_ = {nullptr, nullptr};
    }
    ~GroupTimer() {
        roctxRangePop();
        if (!ev_.first) return;
        if (hipEventRecord(ev_.second, h_->stream) == hipSuccess)
            h_->timed.push_back({ev_.first, ev_.second, cls_});
        else
            h_->event_pool.push_back(ev_);
    }

  private:
    misa_lattice *h_;
    int cls_;
    std::pair<hipEvent_t, hipEvent_t> ev_{nullptr, nullptr};
};

// Sum recorded groups into the totals (synchronises the stream).
hipError_t fold_timing(misa_lattice *h) {
    if (h->timed.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    for (auto &t : h->timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            h->timer_ms[t.cls] += ms;
            h->timer_n[t.cls] += 1;
        }
        h->event_pool.push_back({t.start, t.stop});
    }
    h->timed.clear();
    return hipSuccess;
}

int do_rho(misa_lattice *h) {
    if (h->pending_clear) {
        GroupTimer t(h, MISA_TIMER_RUNAWAY);
        HIPCHK(h, clear_marks(h));
        HIPCHK(h, launch_runaway_clear(h));
        h->pending_clear = false;
    }
    {
        GroupTimer t(h, MISA_TIMER_RUNAWAY);
        HIPCHK(h, launch_runaway_build(h));
    }
    {
        GroupTimer t(h, MISA_TIMER_RHO);
        HIPCHK(h, launch_rho(h));
    }
    {
        GroupTimer t(h, MISA_TIMER_RUNAWAY);
        HIPCHK(h, launch_runaway_rho(h));
    }
    h->pending_clear = true;
    h->rho_valid = true;
    h->force_valid = false;
    return MISA_OK;
}

// Force pass (kick: with the fused second half-kick).  The cell lists and the affected
// list stay alive for the step statistics until finish_force.
int do_force(misa_lattice *h, bool energy, double *energies_dev, bool kick) {
    {
        GroupTimer t(h, MISA_TIMER_FORCE);
        HIPCHK(h, launch_force(h, energy, kick));
    }
    {
        GroupTimer t(h, MISA_TIMER_RUNAWAY);
        HIPCHK(h, launch_runaway_force(h, energy, kick));
    }
    {
        GroupTimer t(h, MISA_TIMER_OTHER);
        if (energy) HIPCHK(h, launch_energy_reduce(h, energies_dev));
    }
    h->force_valid = true;
    return MISA_OK;
}

int finish_force(misa_lattice *h) {
    GroupTimer t(h, MISA_TIMER_RUNAWAY);
    HIPCHK(h, launch_runaway_clear(h));
    h->pending_clear = false;
    return MISA_OK;
}

// One MD step (Fig. 1 in kick-drift-kick form): the kernels of the rho and force
// passes, the run-away path and the integrator, with no host synchronisation.
int step_body(misa_lattice *h, bool last, bool fused, double dt_max, double dx_max) {
    struct StepRange {
        StepRange() { roctxRangePushA("misa:step"); }
        ~StepRange() { roctxRangePop(); }
    } range;
    int rc;
    {
        GroupTimer t(h, MISA_TIMER_KICK);
        HIPCHK(h, launch_kick_drift(h));
    }
    {
        GroupTimer t(h, MISA_TIMER_RUNAWAY);
        HIPCHK(h, launch_rehash(h));
    }
    if ((rc = do_rho(h))) return rc;
    if ((rc = do_force(h, last, nullptr, fused))) return rc;
    {
        GroupTimer t(h, MISA_TIMER_KICK);
        HIPCHK(h, launch_final_kick(h));
    }
    {
        GroupTimer t(h, MISA_TIMER_OTHER);
        HIPCHK(h, launch_dt_update(h, dt_max, dx_max, false));
    }
    if ((rc = finish_force(h))) return rc;  // after the step statistics read the affected list
    if (h->timed.size() > 50000) HIPCHK(h, fold_timing(h));  // bound the event backlog
    return MISA_OK;
}

// Capture one regular step, starting from the current copy of u and v, into
// h->graph_exec[h->parity] (a step ends on the other copy, so consecutive steps
// replay the two graphs in turn).  The capture runs on a private stream (the
// caller's may be the legacy default stream, which cannot capture); the host-side
// flags a step updates, and the current copy, end where they started.
int capture_step(misa_lattice *h, bool fused, double dt_max, double dx_max) {
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int par = h->parity;
    hipStream_t user = h->stream;
    h->stream = h->cap_stream;
    hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    int rc = MISA_OK;
    if (e == hipSuccess) rc = step_body(h, false, fused, dt_max, dx_max);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(h->stream, &graph) : e;
    h->stream = user;
    if (h->parity != par) swap_uv(h);  // nothing ran: the state is still on the copy it started from
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    HIPCHK(h, e2);
    e = hipGraphInstantiate(&h->graph_exec[par], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) h->graph_exec[par] = nullptr;
    HIPCHK(h, e);
    h->graph_dt[par] = dt_max;
    h->graph_dx[par] = dx_max;
    return MISA_OK;
}

}  // namespace

// k_clear_marks lives here: it only zeroes mark words of listed sites.
namespace misa {
void drop_graph(misa_lattice *h) {
    for (hipGraphExec_t &g : h->graph_exec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    ++h->gen;  // a batch's captured step that holds this box goes stale too
}

__global__ void k_clear_marks(Scratch sc) {
    int na = sc.cnt->n_affected;
    na = na < sc.affected_cap ? na : (int)sc.affected_cap;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < na; q += gridDim.x * blockDim.x)
        sc.mark[sc.affected[q] >> 5] = 0u;
}
}  // namespace misa

namespace {
hipError_t clear_marks(misa_lattice *h) {
    hipLaunchKernelGGL(misa::k_clear_marks, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->sc);
    return hipGetLastError();
}
}  // namespace

// ===========================================================================
// C ABI

extern "C" {

const char *misa_last_error(const misa_lattice *h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

int misa_create_lattice(const misa_lattice_desc *d, void *hip_stream, misa_lattice **out) {
    if (!d || !out) return fail(nullptr, MISA_EINVAL, "null descriptor or output pointer");
    *out = nullptr;
    for (int k = 0; k < 3; ++k)
        if (d->n_cells[k] < 1) return fail(nullptr, MISA_EINVAL, "n_cells must be >= 1");
    if (!(d->a > 0) || !(d->rc > 0) || !(d->mass > 0)) return fail(nullptr, MISA_EINVAL, "a, rc and mass must be > 0");
    if (!(d->delta > 0) || !(d->delta < d->a * std::sqrt(3.0) / 4.0))
        return fail(nullptr, MISA_EINVAL, "delta must lie in (0, a sqrt(3)/4)");
    if (d->pair_precision != MISA_FP64 && d->pair_precision != MISA_FP32 && d->pair_precision != MISA_MLP)
        return fail(nullptr, MISA_EINVAL, "pair_precision must be MISA_FP64, MISA_FP32 or MISA_MLP");
    for (int k = 0; k < 3; ++k)
        if (d->periodic[k] != 0 && d->periodic[k] != 1)
            return fail(nullptr, MISA_EINVAL, "periodic must be 1 (or 0, the default) on every axis: only periodic boxes");
    if (d->ntypes != 0 && d->ntypes != 1) return fail(nullptr, MISA_EINVAL, "ntypes must be 1 (or 0, the default)");
    const double R = d->rc + 2.0 * d->delta;
    for (int k = 0; k < 3; ++k)
        if (!(d->n_cells[k] * d->a > 2.0 * R))
            return fail(nullptr, MISA_EINVAL, "box too small: n_cells * a must exceed 2 (rc + 2 delta) on every axis");
    const int64_t ncell = (int64_t)d->n_cells[0] * d->n_cells[1] * d->n_cells[2];
    if (2 * ncell >= (int64_t)INT32_MAX) return fail(nullptr, MISA_EINVAL, "too many sites (max 2^31 - 1)");

    misa_lattice *h = new (std::nothrow) misa_lattice();
    if (!h) return fail(nullptr, MISA_ENOMEM, "host allocation failed");
    h->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&h->device);
    h->use_mlp = d->pair_precision == MISA_MLP;
    h->precision = h->use_mlp ? MISA_FP32 : d->pair_precision;
    h->mass = d->mass;
    Geom &g = h->g;
    g.nx = d->n_cells[0];
    g.ny = d->n_cells[1];
    g.nz = d->n_cells[2];
    g.ntx = (g.nx + TX - 1) / TX;
    g.nty = (g.ny + TY - 1) / TY;
    g.ntz = (g.nz + TZ - 1) / TZ;
    g.ntiles = g.ntx * g.nty * g.ntz;
    g.ntiles_pad = (g.ntiles + 7) / 8 * 8;
    g.nt2[0] = (g.nx + T2X - 1) / T2X;
    g.nt2[1] = (g.ny + T2Y - 1) / T2Y;
    g.nt2[2] = (g.nz + T2Z - 1) / T2Z;
    g.ntiles2 = g.nt2[0] * g.nt2[1] * g.nt2[2];
    g.ntiles2_pad = (g.ntiles2 + 7) / 8 * 8;
    for (int a = 0; a < 3; ++a) {
        g.tshape[a] = a == 0 ? T2X : (a == 1 ? T2Y : T2Z);
        const uint32_t side = (uint32_t)(g.tshape[a] + 2 * HALO);
        g.tdiv[a] = (uint32_t)((0x100000000ull + side - 1) / side);
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) ncu = 0;
        h->n_cu = ncu;
        // one 1024-lane work-group per compute unit (LDS-bound), a multiple of the 8 XCDs
        h->persistent_grid = ncu >= 8 ? ncu / 8 * 8 : 0;
    }
    g.ncell = ncell;
    g.nsites = 2 * ncell;
    g.a = d->a;
    g.inv_a = 1.0 / d->a;
    const int32_t n3[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        g.L[k] = (double)n3[k] * d->a;
        g.inv_L[k] = 1.0 / g.L[k];
    }
    g.rc = d->rc;
    g.rc2 = d->rc * d->rc;
    g.delta2 = d->delta * d->delta;
    g.pre2 = (d->rc * (1.0 + 1e-9)) * (d->rc * (1.0 + 1e-9));
    for (int k = 0; k < 3; ++k) {
        int nc = (int)std::floor(g.L[k] / (d->rc * (1.0 + 1e-9)));
        if (nc < 1) nc = 1;
        g.nc[k] = nc;
        g.inv_cs[k] = (double)nc / g.L[k];
    }
    if ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] >= (int64_t)INT32_MAX) {
        delete h;
        return fail(nullptr, MISA_EINVAL, "too many coarse cells");
    }
    g.reach = (d->rc + d->delta) / d->a;
    g.win = (int)std::ceil(2.0 * g.reach + 0.5);
    for (int k = 0; k < 3; ++k)
        if (g.win > n3[k]) {
            delete h;
            return fail(nullptr, MISA_EINVAL, "box too small for the run-away search window");
        }
    h->rcap = d->runaway_capacity > 0 ? d->runaway_capacity : std::max<int64_t>(16384, g.nsites / 1024);
    if (h->rcap > (int64_t)1 << 28) {
        delete h;
        return fail(nullptr, MISA_EINVAL, "runaway_capacity too large");
    }

    // Neighbor Offset Index per parity
    std::vector<CanonOffset> st[2] = {enumerate_offsets(d->a, R, 0), enumerate_offsets(d->a, R, 1)};
    if (st[0].size() != st[1].size() || st[0].size() > (size_t)KMAX) {
        delete h;
        return fail(nullptr, MISA_EINVAL, "stencil larger than the kernels support (rc + 2 delta too large)");
    }
    h->K = (int)st[0].size();
    h->d_min = h->K > 0 ? std::sqrt(st[0][0].d2) : 0.0;  // offsets are sorted nearest first
    {
        int kin = 0;
        while (kin < h->K && st[0][kin].d2 < d->rc * d->rc) ++kin;
        h->K_in = kin;
        if (kin < h->K) {  // |u| bound below which entries kin.. cannot reach rc (1e-3 A margin for float32)
            const double u_cut = 0.5 * (std::sqrt(st[0][kin].d2) - d->rc) - 1e-3;
            h->u_cut2 = u_cut > 0.0 ? (float)(u_cut * u_cut) : -1.f;
        }
    }
    h->stencil_canon.resize(2 * h->K * 3);
    std::vector<StencilEntry<double>> s64(2 * KMAX), s64p(2 * KMAX);
    std::vector<StencilEntry<float>> s32(2 * KMAX), s32p(2 * KMAX);
    NearTab ng{}, nh{};
    ng.rc2 = nh.rc2 = d->rc * d->rc;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 64; ++k) ng.thr2[p][k] = nh.thr2[p][k] = -1.f;
    auto near_thr = [&](const CanonOffset &o) {
        const double t = 0.5 * (d->rc - std::sqrt(o.d2) - (double)NEAR_MARGIN);
        return t > 0.0 ? (float)(t * t) : -1.f;
    };
    for (int p = 0; p < 2; ++p)  // |o_k| is the same for both parities
        for (int k = 0; k < h->K && k < 64; ++k) ng.thr2[p][k] = near_thr(st[0][k]);
    auto near_of = [&](const CanonOffset &o, int p) {
        const int pn = ((p + o.dX) % 2 + 2) % 2;
        return NearEntry{(int32_t)o.dX, (int32_t)o.dY, (int32_t)o.dZ, 0, o.dX * 0.5 * d->a,
                         (o.dY + 0.5 * pn - 0.5 * p) * d->a, (o.dZ + 0.5 * pn - 0.5 * p) * d->a, 0.0};
    };
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < h->K; ++k) {
            const CanonOffset &o = st[p][k];
            const int pn = ((p + o.dX) % 2 + 2) % 2;
            const int dcx = (p + o.dX - pn) / 2, dcy = o.dY, dcz = o.dZ;
            if (std::abs(dcx) > HALO || std::abs(dcy) > HALO || std::abs(dcz) > HALO) {
                delete h;
                return fail(nullptr, MISA_EINVAL, "stencil reaches beyond the LDS halo (rc + 2 delta too large)");
            }
            const int lds = (pn - p) * PZ * PY * PX + (dcz * PY + dcy) * PX + dcx;
            const double ox = o.dX * 0.5 * d->a;
            const double oy = (o.dY + 0.5 * pn - 0.5 * p) * d->a;
            const double oz = (o.dZ + 0.5 * pn - 0.5 * p) * d->a;
            s64[p * KMAX + k] = StencilEntry<double>{lds, 0, ox, oy, oz};
            s32[p * KMAX + k] = StencilEntry<float>{lds, (float)ox, (float)oy, (float)oz};
            const int lds2 = (pn - p) * P2Z * P2Y * P2X + (dcz * P2Y + dcy) * P2X + dcx;
            s32p[p * KMAX + k] = StencilEntry<float>{lds2, (float)ox, (float)oy, (float)oz};
            s64p[p * KMAX + k] = StencilEntry<double>{lds2, 0, ox, oy, oz};
            ng.st[p][k] = near_of(o, p);
            int64_t *c = &h->stencil_canon[(p * h->K + k) * 3];
            c[0] = o.dX;
            c[1] = o.dY;
            c[2] = o.dZ;
        }
    // Half stencil: the entries whose lattice offset points into the forward half
    // space (dZ > 0, or dZ = 0 and dY > 0, or dZ = dY = 0 and dX > 0), grouped by
    // phase (dZ, partner parity != own) and nearest first inside a phase (the
    // stable sort keeps the distance order of st).
    std::vector<StencilEntry<float>> sh(2 * KMAX, StencilEntry<float>{0, 0.f, 0.f, 0.f});
    std::vector<int32_t> hmeta(2 * HALF_META, 0);
    for (int p = 0; p < 2; ++p) {
        std::vector<std::pair<int, int>> fw;  // (phase, k)
        for (int k = 0; k < h->K; ++k) {
            const CanonOffset &o = st[p][k];
            const bool forward = o.dZ > 0 || (o.dZ == 0 && (o.dY > 0 || (o.dY == 0 && o.dX > 0)));
            if (!forward) continue;
            const int pn = ((p + o.dX) % 2 + 2) % 2;
            fw.push_back({2 * (int)o.dZ + (pn != p ? 1 : 0), k});
        }
        std::stable_sort(fw.begin(), fw.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
            return x.first < y.first;
        });
        int32_t *m = &hmeta[p * HALF_META];
        for (int q = 0, n = 0; q <= HALF_PHASES; ++q) {
            while (n < (int)fw.size() && fw[n].first < q) ++n;
            m[q] = n;
        }
        for (size_t i = 0; i < fw.size(); ++i) {
            const CanonOffset &o = st[p][fw[i].second];
            const int pn = ((p + o.dX) % 2 + 2) % 2;
            const int dcx = (p + o.dX - pn) / 2, dcy = o.dY, dcz = o.dZ;
            const int lds = (pn - p) * HFZ * HFY * HFX + (dcz * HFY + dcy) * HFX + dcx;
            sh[p * KMAX + i] = StencilEntry<float>{lds, (float)(o.dX * 0.5 * d->a),
                                                   (float)((o.dY + 0.5 * pn - 0.5 * p) * d->a),
                                                   (float)((o.dZ + 0.5 * pn - 0.5 * p) * d->a)};
            nh.st[p][i] = near_of(o, p);
            if (i < 64) nh.thr2[p][i] = near_thr(o);
            if (o.d2 < d->rc * d->rc) ++m[8 + fw[i].first];
        }
        h->half_entries = std::max(h->half_entries, (int)m[HALF_PHASES]);
    }

    // scratch
    Scratch &sc = h->sc;
    const int64_t rcap = h->rcap;
    const int64_t ncc = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    sc.cs_nblk = (int32_t)((ncc + CS_CHUNK - 1) / CS_CHUNK);
    const int64_t ncc_pad = (int64_t)sc.cs_nblk * CS_CHUNK;
    // lattice atoms within rc of a run-away, plus those of the float32 gather form with a
    // pair inside the cut-off band (about one atom in 10^3 at 300 K)
    sc.affected_cap = std::min<int64_t>(g.nsites, 128 * rcap + g.nsites / 16 + 64);
    {
        const int64_t per_blk = (int64_t)MARK_THREADS * MARK_WORDS;
        sc.mark_nblk = (int32_t)(((g.nsites + 31) / 32 + per_blk - 1) / per_blk);
        sc.mark_nwords = sc.mark_nblk * per_blk;
    }
    auto bail = [&](hipError_t e) {
        std::string m = std::string("device allocation failed: ") + hipGetErrorString(e);
        misa_destroy_lattice(h);
        return fail(nullptr, MISA_ENOMEM, m);
    };
    hipError_t e;
#define ALLOC(ptr, n)                          \
    if ((e = dev_alloc(&(ptr), (n))) != hipSuccess) return bail(e);
    ALLOC(h->st64, 2 * KMAX);
    ALLOC(h->st32, 2 * KMAX);
    ALLOC(h->st32p, 2 * KMAX);
    ALLOC(h->st64p, 2 * KMAX);
    ALLOC(h->sth, 2 * KMAX);
    ALLOC(h->near_g, 1);
    ALLOC(h->near_h, 1);
    ALLOC(h->hmeta, 2 * HALF_META);
    ALLOC(sc.cnt, 1);
    ALLOC(sc.scal, 8);
    // per-tile partials of any tiling a batch may choose for this box
    int64_t max_tiles = std::max<int64_t>(g.ntiles_pad, g.ntiles2_pad);
    for (int sh = 0; sh < N_TILE_SHAPES; ++sh) {
        const int *t = TILE_SHAPES[sh];
        const int64_t n = (int64_t)((g.nx + t[0] - 1) / t[0]) * ((g.ny + t[1] - 1) / t[1]) * ((g.nz + t[2] - 1) / t[2]);
        max_tiles = std::max<int64_t>(max_tiles, (n + 7) / 8 * 8);
    }
    ALLOC(sc.part, 2 * max_tiles + 2 * 1024);
    ALLOC(sc.l_site, rcap);
    ALLOC(sc.l_id, rcap);
    ALLOC(sc.l_x, rcap);
    ALLOC(sc.l_y, rcap);
    ALLOC(sc.l_z, rcap);
    ALLOC(sc.l_vx, rcap);
    ALLOC(sc.l_vy, rcap);
    ALLOC(sc.l_vz, rcap);
    ALLOC(sc.cand, rcap);
    ALLOC(sc.settled, rcap);
    ALLOC(sc.sortbuf, next_pow2(rcap));
    ALLOC(sc.skey, rcap);
    ALLOC(sc.sidx, rcap);
    ALLOC(sc.cell_n, ncc_pad);
    ALLOC(sc.cell_s, ncc_pad + 1);
    ALLOC(sc.cs_blk, sc.cs_nblk);
    ALLOC(sc.srx, rcap);
    ALLOC(sc.sry, rcap);
    ALLOC(sc.srz, rcap);
    ALLOC(sc.cellq, rcap);
    ALLOC(sc.sfp, rcap);
    ALLOC(sc.loneq, rcap);
    ALLOC(sc.sorder, rcap);
    ALLOC(sc.mark, sc.mark_nwords);
    ALLOC(sc.mark_blk, sc.mark_nblk);
    ALLOC(sc.mark_off, sc.mark_nblk);
    ALLOC(sc.affected, sc.affected_cap);
    ALLOC(sc.aff_v2, sc.affected_cap);
    ALLOC(sc.aff_e, sc.affected_cap);
    ALLOC(sc.part_kick, 2 * std::max<int64_t>(max_tiles, 8));
#undef ALLOC
    if ((e = hipMemcpy(h->st64, s64.data(), sizeof(StencilEntry<double>) * 2 * KMAX, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->st32, s32.data(), sizeof(StencilEntry<float>) * 2 * KMAX, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->st32p, s32p.data(), sizeof(StencilEntry<float>) * 2 * KMAX, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->st64p, s64p.data(), sizeof(StencilEntry<double>) * 2 * KMAX, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->sth, sh.data(), sizeof(StencilEntry<float>) * 2 * KMAX, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->near_g, &ng, sizeof(NearTab), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->near_h, &nh, sizeof(NearTab), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(h->hmeta, hmeta.data(), sizeof(int32_t) * 2 * HALF_META, hipMemcpyHostToDevice)) ||
        (e = hipMemset(sc.cnt, 0, sizeof(Counters))) || (e = hipMemset(sc.scal, 0, 8 * sizeof(double))) ||
        (e = hipMemset(sc.cell_n, 0, sizeof(int32_t) * (size_t)ncc_pad)) ||
        (e = hipMemset(sc.mark, 0, sizeof(uint32_t) * (size_t)sc.mark_nwords)) ||
        (e = hipDeviceSynchronize())) {
        std::string m = std::string("device initialisation failed: ") + hipGetErrorString(e);
        misa_destroy_lattice(h);
        return fail(nullptr, MISA_EHIP, m);
    }
    {
        void *sp = nullptr;  // once per device, with the device current (misa_set_state_noalloc reports failures)
        (void)scratch_address(h->device, &sp);
    }
    h->half.st = h->sth;
    h->half.meta = h->hmeta;
    h->half_fits = g.nx % (2 * T2X) == 0 && g.ny % (2 * T2Y) == 0 && g.nz % (2 * T2Z) == 0;
    *out = h;
    return MISA_OK;
}

int misa_destroy_lattice(misa_lattice *h) {
    if (!h) return MISA_OK;
    if (h->stream)
        (void)hipStreamSynchronize(h->stream);
    else
        (void)hipDeviceSynchronize();
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    void *ptrs[] = {h->st64, h->st32, h->st32p, h->st64p, h->near_g, h->near_h, h->sth, h->hmeta, h->lds32.lf, h->lds32.lg, h->fwin64.recs, h->fwin64.band, h->rwin64.recs, h->rwin64.band, h->lds32h.f,
                    h->lds32h.force, h->t64.f, h->t64.force, h->t64.phi, h->t64.emb, h->t64.force6, h->t32.force6, h->t32.f, h->t32.force,
                    h->t32.phi, h->t32.emb, h->sc.cnt, h->sc.scal, h->sc.part, h->sc.l_site, h->sc.l_id, h->sc.l_x,
                    h->sc.l_y, h->sc.l_z, h->sc.l_vx, h->sc.l_vy, h->sc.l_vz, h->sc.cand, h->sc.settled,
                    h->sc.sortbuf, h->sc.skey, h->sc.sidx, h->sc.cell_n, h->sc.cell_s, h->sc.cs_blk,
                    h->sc.srx, h->sc.sry, h->sc.srz, h->sc.cellq, h->sc.loneq, h->sc.sorder, h->sc.sfp, h->sc.mark,
                    h->sc.mark_blk, h->sc.mark_off, h->sc.affected, h->sc.aff_v2, h->sc.aff_e, h->sc.part_kick, h->staging,
                    h->mlp.p[0], h->mlp.p[1], h->mlp.p[2], h->mlp.w2b[0], h->mlp.w2b[1], h->mlp.w2b[2],
                    h->pairbuf};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &t : h->timed) h->event_pool.push_back({t.start, t.stop});
    for (auto &ev : h->event_pool) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    delete h;
    return MISA_OK;
}

int misa_state_bytes(const misa_lattice *h, int64_t *bytes) {
    if (!h || !bytes) return fail(nullptr, MISA_EINVAL, "null argument");
    *bytes = carve(const_cast<misa_lattice *>(h), nullptr, nullptr);
    return MISA_OK;
}

int misa_bind_state(misa_lattice *h, void *device_ptr, int64_t bytes) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    const int64_t need = carve(h, nullptr, nullptr);
    if (!device_ptr || bytes < need) return fail(h, MISA_EINVAL, "state buffer missing or smaller than misa_state_bytes");
    if (((uintptr_t)device_ptr & 255u) != 0) return fail(h, MISA_EINVAL, "state buffer must be 256-byte aligned");
    h->state_ptr = device_ptr;
    h->state_bytes = bytes;
    carve(h, (char *)device_ptr, &h->S, &h->alt);
    h->parity = 0;
    h->state_bound = true;
    drop_graph(h);
    h->state_set = h->rho_valid = h->force_valid = false;
    return MISA_OK;
}

namespace {
// Bands of table segments for a persistent float64 pass with room for cap LDS records
// (BandWin64): per stencil entry the band around its shell distance (entries past rc:
// the top band).  Returns the bands (in LDS order) and the records they take, the zero
// record included.
int shell_bands(misa_lattice *h, const misa_table &f, int nseg, int cap, std::vector<int2> &bands,
                std::vector<int4> &bandv, double &halfwidth) {
    std::vector<StencilEntry<double>> st(2 * KMAX);
    HIPCHK(h, hipMemcpy(st.data(), h->st64p, sizeof(StencilEntry<double>) * 2 * KMAX, hipMemcpyDeviceToHost));
    auto seg_lo = [&](double r) { return std::max(0, std::min(nseg, (int)std::floor((r - f.x0) / f.dx))); };
    auto seg_hi = [&](double r) { return std::max(0, std::min(nseg, (int)std::ceil((r - f.x0) / f.dx))); };
    std::vector<double> shells;  // distinct shell distances within rc
    for (int k = 0; k < h->K; ++k) {
        const StencilEntry<double> &e = st[k];
        const double d = std::sqrt(e.ox * e.ox + e.oy * e.oy + e.oz * e.oz);
        if (d >= h->g.rc) continue;
        bool seen = false;
        for (double c : shells) seen = seen || std::fabs(c - d) < 1e-9;
        if (!seen) shells.push_back(d);
    }
    std::sort(shells.begin(), shells.end());
    // bands [a, b) for half-width w, merged, the last reaching nseg; records incl. the zero one
    auto bands_for = [&](double w, std::vector<int2> &out) {
        std::vector<int2> b;
        for (double c : shells) b.push_back(make_int2(seg_lo(c - w), seg_hi(c + w)));
        b.push_back(make_int2(seg_lo(h->g.rc - w), nseg));
        std::sort(b.begin(), b.end(), [](int2 x, int2 y) { return x.x < y.x; });
        out.clear();
        for (const int2 &x : b) {
            if (!out.empty() && x.x <= out.back().y)
                out.back().y = std::max(out.back().y, x.y);
            else
                out.push_back(x);
        }
        out.back().y = nseg;
        int n = 1;
        for (const int2 &x : out) n += x.y - x.x;
        return n;
    };
    halfwidth = 0.0;
    if (nseg + 1 <= cap) {
        bands.assign(1, make_int2(0, nseg));
    } else {
        double lo = 0.0, hi = 2.0 * h->g.rc;  // widest half-width whose bands fit
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (bands_for(mid, bands) <= cap) lo = mid;
            else hi = mid;
        }
        if (bands_for(lo, bands) > cap) return fail(h, MISA_EINVAL, "float64 table bands exceed their LDS records");
        halfwidth = lo;
    }
    std::vector<int> base;
    int n = 0;
    for (const int2 &b : bands) {
        base.push_back(n);
        n += b.y - b.x;
    }
    bandv.assign(2 * KMAX, make_int4(0, 0, 0, 0));
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < h->K; ++k) {
            const StencilEntry<double> &e = st[p * KMAX + k];
            const double d = std::sqrt(e.ox * e.ox + e.oy * e.oy + e.oz * e.oz);
            const int sd = seg_lo(std::min(d, h->g.rc));
            size_t bi = bands.size() - 1;
            for (size_t i = 0; i < bands.size(); ++i)
                if (sd >= bands[i].x && sd < bands[i].y) bi = i;
            const bool top = bi + 1 == bands.size();
            bandv[p * KMAX + k] = make_int4(bands[bi].x, bands[bi].y - bands[bi].x + (top ? 1 : 0), base[bi], 0);
        }
    return MISA_OK;
}

// The LDS records of the persistent float64 passes (BandWin64): force records (f' and
// phi' quadratics, 3 double2) and density records (f cubic, 2 double2).
int build_windows64(misa_lattice *h, const misa_table &f, const std::vector<SegCoef> &sf,
                    const std::vector<SegCoef> &sp) {
    const int nseg = (int)sf.size();
    for (int which = 0; which < 2; ++which) {
        BandWin64 &W = which == 0 ? h->fwin64 : h->rwin64;
        (void)hipFree(W.recs);
        (void)hipFree(W.band);
        W = BandWin64{};
        std::vector<int2> bands;
        std::vector<int4> bandv;
        double w = 0.0;
        const int rc = shell_bands(h, f, nseg, which == 0 ? FWIN64_MAX + 1 : RWIN64_MAX, bands, bandv, w);
        if (rc) return rc;
        std::vector<double2> recs;
        for (const int2 &b : bands)
            for (int s = b.x; s < b.y; ++s) {
                if (which == 0) {
                    recs.push_back(make_double2(sf[s].d0, sf[s].d1));
                    recs.push_back(make_double2(sf[s].d2, sp[s].d0));
                    recs.push_back(make_double2(sp[s].d1, sp[s].d2));
                } else {
                    recs.push_back(make_double2(sf[s].c0, sf[s].c1));
                    recs.push_back(make_double2(sf[s].c2, sf[s].c3));
                }
            }
        const int per = which == 0 ? 3 : 2;
        for (int i = 0; i < per; ++i) recs.push_back(make_double2(0.0, 0.0));  // segment nseg
        HIPCHK(h, dev_alloc(&W.recs, (int64_t)recs.size()));
        HIPCHK(h, dev_alloc(&W.band, (int64_t)(2 * KMAX)));
        HIPCHK(h, hipMemcpy(W.recs, recs.data(), sizeof(double2) * recs.size(), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(W.band, bandv.data(), sizeof(int4) * 2 * KMAX, hipMemcpyHostToDevice));
        W.nrec = (int32_t)(recs.size() / per);
        W.halfwidth = w;
    }
    return MISA_OK;
}
}  // namespace

namespace {
int set_tables_impl(misa_lattice *h, const misa_table *f, const misa_table *phi, const misa_table *emb);
}

int misa_set_potential_tables(misa_lattice *h, const misa_table *f, const misa_table *phi, const misa_table *emb) {
    const int rc = set_tables_impl(h, f, phi, emb);
    if (rc) return rc;
    const misa_table *t3[3] = {f, phi, emb};
    for (int i = 0; i < 3; ++i) {
        h->tab_y[i].assign(t3[i]->y, t3[i]->y + t3[i]->n);
        h->tab[i] = *t3[i];
        h->tab[i].y = h->tab_y[i].data();
    }
    return MISA_OK;
}

}  // extern "C"

namespace {
int set_tables_impl(misa_lattice *h, const misa_table *f, const misa_table *phi, const misa_table *emb) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    const misa_table *t3[3] = {f, phi, emb};
    for (const misa_table *t : t3) {
        if (!t || !t->y) return fail(h, MISA_EINVAL, "null table");
        if (t->n < 8 || !(t->dx > 0) || !std::isfinite(t->x0)) return fail(h, MISA_EINVAL, "tables need n >= 8 and dx > 0");
        for (int k = 0; k < t->n; ++k)
            if (!std::isfinite(t->y[k])) return fail(h, MISA_EINVAL, "non-finite table sample");
    }
    if (f->x0 != phi->x0 || f->dx != phi->dx || f->n != phi->n)
        return fail(h, MISA_EINVAL, "f and phi must share one grid");
    if (f->x0 < 0.0 || f->x0 + (f->n - 1) * f->dx < h->g.rc * (1.0 - 1e-12))
        return fail(h, MISA_EINVAL, "f/phi grid must start at x0 >= 0 and reach rc");
    const std::vector<SegCoef> sf = segments(*f), sp = segments(*phi), se = segments(*emb);
    int rc = upload_tables<double>(h, h->t64, sf, sp, se, *f, *emb);
    if (rc) return rc;
    rc = upload_tables<float>(h, h->t32, sf, sp, se, *f, *emb);
    if (rc) return rc;
    // LDS windows for the persistent float32 kernels (gather passes: 6143 linear
    // segments; half-stencil passes, which also hold accumulators in LDS: 2879 cubic /
    // quadratic segments): two slotted
    // atoms are never closer than the nearest-neighbour site distance minus 2 delta.
    for (int wi = 0; wi < 2; ++wi) {
        LdsTables &W = wi == 0 ? h->lds32 : h->lds32h;
        (void)hipFree(W.f);
        (void)hipFree(W.force);
        (void)hipFree(W.lf);
        (void)hipFree(W.lg);
        W = LdsTables{};
        const double delta = std::sqrt(h->g.delta2);
        const double r_lo = h->d_min - 2.0 * delta - 2.0 * f->dx;
        int64_t k0 = (int64_t)std::floor((r_lo - f->x0) / f->dx);
        k0 = std::max<int64_t>(0, std::min<int64_t>(k0, f->n - 2));
        const double x_last = f->x0 + (f->n - 1) * f->dx;
        const double r0 = std::max(f->x0 + k0 * f->dx, 1e-3);
        const double q0 = r0 * r0, q1 = x_last * x_last;
        const int64_t nwin = (wi == 0 ? LDS_TAB_SEGS : HALF_TAB_SEGS) - 1;  // + 1: the zero record after the window
        const double hq = (q1 - q0) / (double)nwin;
        // the float64 spline (value and d/dr) of a source table at r
        auto spline = [&](const std::vector<SegCoef> &S, double r, double &v, double &d) {
            const double p = (r - f->x0) / f->dx;
            int64_t k = (int64_t)std::floor(p);
            k = std::max<int64_t>(0, std::min<int64_t>(k, f->n - 2));
            const double t = p - (double)k;
            const SegCoef &c = S[k];
            v = ((c.c3 * t + c.c2) * t + c.c1) * t + c.c0;
            d = (c.d2 * t + c.d1) * t + c.d0;
        };
        if (wi == 0) {  // gather window: linear records between the spline's values at the q nodes
            std::vector<float2> lf(nwin);
            std::vector<float4> lg(nwin);
            double fv0 = 0.0, gf0 = 0.0, gp0 = 0.0;
            for (int64_t s = 0; s <= nwin; ++s) {
                const double r = std::sqrt(q0 + (double)s * hq);
                double fv, fd, pv, pd;
                spline(sf, r, fv, fd);
                spline(sp, r, pv, pd);
                const double gf = fd / r, gp = pd / r;
                if (s > 0) {
                    lf[s - 1] = make_float2((float)fv0, (float)(fv - fv0));
                    lg[s - 1] = make_float4((float)gf0, (float)(gf - gf0), (float)gp0, (float)(gp - gp0));
                }
                fv0 = fv;
                gf0 = gf;
                gp0 = gp;
            }
            HIPCHK(h, dev_alloc(&W.lf, nwin));
            HIPCHK(h, dev_alloc(&W.lg, nwin));
            HIPCHK(h, hipMemcpy(W.lf, lf.data(), sizeof(float2) * nwin, hipMemcpyHostToDevice));
            HIPCHK(h, hipMemcpy(W.lg, lg.data(), sizeof(float4) * nwin, hipMemcpyHostToDevice));
        } else {  // half-stencil window: cubic value and quadratic force records
            std::vector<Q4<float>> wf(nwin);
            std::vector<FRec32> wr(nwin);
            for (int64_t s = 0; s < nwin; ++s) {
                double fv[4], gf[3], gp[3];
                for (int i = 0; i < 4; ++i) {  // f at t = 0, 1/3, 2/3, 1
                    const double r = std::sqrt(q0 + ((double)s + i / 3.0) * hq);
                    double d;
                    spline(sf, r, fv[i], d);
                }
                for (int i = 0; i < 3; ++i) {  // f'/r and phi'/r at t = 0, 1/2, 1
                    const double r = std::sqrt(q0 + ((double)s + 0.5 * i) * hq);
                    double v, d;
                    spline(sf, r, v, d);
                    gf[i] = d / r;
                    spline(sp, r, v, d);
                    gp[i] = d / r;
                }
                // Newton forward differences -> power basis in t
                const double d1 = fv[1] - fv[0], d2 = fv[2] - 2.0 * fv[1] + fv[0],
                             d3 = fv[3] - 3.0 * fv[2] + 3.0 * fv[1] - fv[0];
                wf[s] = {(float)fv[0], (float)(3.0 * d1 - 1.5 * d2 + d3), (float)(4.5 * d2 - 4.5 * d3),
                         (float)(4.5 * d3)};
                auto quad = [](const double y[3], double &a0, double &a1, double &a2) {
                    const double e1 = y[1] - y[0], e2 = y[2] - 2.0 * y[1] + y[0];
                    a0 = y[0];
                    a1 = 2.0 * e1 - e2;
                    a2 = 2.0 * e2;
                };
                double f0, f1, f2, p0, p1, p2;
                quad(gf, f0, f1, f2);
                quad(gp, p0, p1, p2);
                wr[s].a = make_float2((float)f0, (float)f1);
                wr[s].b = make_float2((float)f2, (float)p0);
                wr[s].c = make_float2((float)p1, (float)p2);
            }
            HIPCHK(h, dev_alloc(&W.f, nwin));
            HIPCHK(h, dev_alloc(&W.force, nwin));
            HIPCHK(h, hipMemcpy(W.f, wf.data(), sizeof(Q4<float>) * nwin, hipMemcpyHostToDevice));
            HIPCHK(h, hipMemcpy(W.force, wr.data(), sizeof(FRec32) * nwin, hipMemcpyHostToDevice));
        }
        W.k0 = (int32_t)k0;
        W.nwin = (int32_t)nwin;
        W.inv_hq = (float)(1.0 / hq);
        W.pcq = (float)(-q0 / hq);
        W.usable = q1 > q0;
        W.node_cut = std::fabs(x_last - h->g.rc) <= 1e-12 * h->g.rc;
    }
    // LDS records of the persistent float64 passes (BandWin64)
    if (h->precision == MISA_FP64 && !h->use_mlp) {
        const int rc = build_windows64(h, *f, sf, sp);
        if (rc) return rc;
    }
    h->tables_set = true;
    h->rho_valid = h->force_valid = false;
    drop_graph(h);
    return MISA_OK;
}
}  // namespace

extern "C" {

}  // extern "C"

namespace {
// Placement of n atoms from device arrays xd, vd: cand (n bids) and bad (one
// counter) are device scratch the caller provides; done(rc) releases whatever
// the caller allocated and returns rc.
template <class Done>
int place_atoms(misa_lattice *h, const double *xd, const double *vd, int64_t n, int32_t *cand, uint32_t *bad,
                Done done) {
    Counters c{};
    hipError_t e = hipMemcpy(h->sc.cnt, &c, sizeof(c), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_fill_u32(h, bad, 0u, 1);
    if (e == hipSuccess) e = launch_place(h, xd, vd, n, cand, bad);
    uint32_t nbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&c, h->sc.cnt, sizeof(c), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return done(fail(h, MISA_EHIP, std::string("placement: ") + hipGetErrorString(e)));
    if (nbad) return done(fail(h, MISA_EINVAL, "non-finite position or velocity"));
    const int64_t R = c.n_leave;
    if (R > h->rcap)
        return done(fail(h, MISA_EOVERFLOW, "more atoms off their sites (" + std::to_string(R) +
                                                ") than the run-away capacity (" + std::to_string(h->rcap) + ")"));
    // the atoms left without a slot become the run-away list in ascending id (the
    // leaver sort and compaction; no bid succeeds, every slot they could claim is taken)
    e = launch_rehash(h);
    const State &S = h->S;
    if (e == hipSuccess && R > 0) {
        e = hipMemsetAsync(S.r_fx, 0, 8 * R, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(S.r_fy, 0, 8 * R, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(S.r_fz, 0, 8 * R, h->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->sc.scal, 0, 8 * sizeof(double), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->sc.mark, 0, sizeof(uint32_t) * (size_t)h->sc.mark_nwords, h->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(h->sc.cell_n, 0, sizeof(int32_t) * (size_t)h->sc.cs_nblk * CS_CHUNK, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return done(fail(h, MISA_EHIP, std::string("placement: ") + hipGetErrorString(e)));
    h->n_atoms = n;
    h->steps_done = 0;
    h->state_set = true;
    return done(MISA_OK);
}

int check_set_state(misa_lattice *h, const double *x, const double *v, int64_t n) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (!h->state_bound) return fail(h, MISA_ESTATE, "no state buffer bound (misa_bind_state)");
    if (n < 0 || n >= (int64_t)INT32_MAX) return fail(h, MISA_EINVAL, "atom count out of range");
    if (n > 0 && (!x || !v)) return fail(h, MISA_EINVAL, "null positions or velocities");
    return MISA_OK;
}
}  // namespace

extern "C" {

int misa_set_state_ids(misa_lattice *h, const double *x, const double *v, const int64_t *ids, int64_t n) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (n < 0 || (n > 0 && (!x || !v || !ids))) return fail(h, MISA_EINVAL, "need x, v and ids for n_atoms > 0");
    // rows in id order; the ids must name every atom once
    std::vector<double> xs((size_t)3 * n), vs((size_t)3 * n);
    std::vector<char> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t id = ids[i];
        if (id < 0 || id >= n || seen[(size_t)id])
            return fail(h, MISA_EINVAL, "ids must be a permutation of 0 .. n_atoms - 1");
        seen[(size_t)id] = 1;
        for (int k = 0; k < 3; ++k) {
            xs[(size_t)3 * id + k] = x[3 * i + k];
            vs[(size_t)3 * id + k] = v[3 * i + k];
        }
    }
    return misa_set_state(h, n ? xs.data() : x, n ? vs.data() : v, n, MISA_HOST);
}

int misa_set_state(misa_lattice *h, const double *x, const double *v, int64_t n, int where) {
    int rc = check_set_state(h, x, v, n);
    if (rc) return rc;
    if (where != MISA_HOST && where != MISA_DEVICE) return fail(h, MISA_EINVAL, "bad memory kind");
    // Placement runs on the device (launch_place): host arrays are uploaded first.
    // Temporary device memory: x, v (host input only), the bid of every atom and a flag.
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->state_set = false;  // until the new state is complete
    h->rho_valid = h->force_valid = h->pending_clear = false;
    const int64_t nn = std::max<int64_t>(n, 1);
    const size_t xv_bytes = where == MISA_HOST ? 2 * sizeof(double) * 3 * (size_t)nn : 0;
    const size_t bytes = xv_bytes + sizeof(int32_t) * (size_t)nn + 256;
    char *tmp = nullptr;
    HIPCHK(h, hipMalloc((void **)&tmp, bytes));
    auto done = [&](int rc) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(tmp);
        return rc;
    };
    const double *xd = x, *vd = v;
    if (where == MISA_HOST && n > 0) {
        double *xs = (double *)tmp, *vs = xs + 3 * nn;
        hipError_t e = hipMemcpy(xs, x, sizeof(double) * 3 * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(vs, v, sizeof(double) * 3 * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return done(fail(h, MISA_EHIP, std::string("upload: ") + hipGetErrorString(e)));
        xd = xs;
        vd = vs;
    }
    int32_t *cand = (int32_t *)(tmp + xv_bytes);
    uint32_t *bad = (uint32_t *)(tmp + xv_bytes + sizeof(int32_t) * (size_t)nn);
    return place_atoms(h, xd, vd, n, cand, bad, done);
}

int misa_set_state_noalloc(misa_lattice *h, const double *x, const double *v, int64_t n) {
    int rc = check_set_state(h, x, v, n);
    if (rc) return rc;
    if (n > MISA_NOALLOC_MAX_ATOMS)
        return fail(h, MISA_EINVAL, "misa_set_state_noalloc: more than MISA_NOALLOC_MAX_ATOMS (" +
                                        std::to_string((long long)MISA_NOALLOC_MAX_ATOMS) + ") atoms");
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if ((int)g_scratch_addr.size() > h->device) base = g_scratch_addr[h->device];
    }
    if (!base) return fail(h, MISA_EHIP, "misa_set_state_noalloc: no device address for the scratch array");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->state_set = false;  // until the new state is complete
    h->rho_valid = h->force_valid = h->pending_clear = false;
    int32_t *cand = (int32_t *)base;
    uint32_t *bad = (uint32_t *)base + MISA_NOALLOC_MAX_ATOMS;
    auto done = [&](int rc2) {
        (void)hipStreamSynchronize(h->stream);
        return rc2;
    };
    return place_atoms(h, x, v, n, cand, bad, done);
}

}  // extern "C"

namespace {
// Checkpoint blob: this header, then the whole bound state buffer (both copies of u
// and v, forces, densities, slots and the run-away list) as the handle holds it.
struct CkptHeader {
    char magic[8];  // "MISACKP1"
    int32_t precision, use_mlp;
    int32_t n_cells[3], parity;
    double a, rc, delta2, mass;
    int64_t rcap, n_atoms, steps_done, state_bytes;
    uint64_t tables_hash;
    int32_t rho_valid, force_valid;
    Counters cnt;
    double scal[8];
};
constexpr char CKPT_MAGIC[8] = {'M', 'I', 'S', 'A', 'C', 'K', 'P', '1'};

// FNV-1a over the three sampled tables (grids and samples) of the last misa_set_potential_tables.
uint64_t tables_hash(const misa_lattice *h) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) x = (x ^ c[i]) * 1099511628211ull;
    };
    for (int i = 0; i < 3; ++i) {
        mix(&h->tab[i].x0, sizeof(double));
        mix(&h->tab[i].dx, sizeof(double));
        mix(h->tab_y[i].data(), sizeof(double) * h->tab_y[i].size());
    }
    return x;
}
}  // namespace

extern "C" {

int misa_checkpoint_bytes(const misa_lattice *h, int64_t *bytes) {
    if (!h || !bytes) return fail(nullptr, MISA_EINVAL, "null argument");
    *bytes = (int64_t)sizeof(CkptHeader) + carve(const_cast<misa_lattice *>(h), nullptr, nullptr);
    return MISA_OK;
}

int misa_save_checkpoint(misa_lattice *h, void *host_out, int64_t bytes) {
    int rc = check_ready(h, true);
    if (rc) return rc;
    const int64_t sb = carve(h, nullptr, nullptr);
    if (!host_out || bytes < (int64_t)sizeof(CkptHeader) + sb)
        return fail(h, MISA_EINVAL, "checkpoint buffer missing or smaller than misa_checkpoint_bytes");
    CkptHeader hd{};
    std::memcpy(hd.magic, CKPT_MAGIC, 8);
    hd.precision = h->precision;
    hd.use_mlp = h->use_mlp;
    hd.n_cells[0] = h->g.nx;
    hd.n_cells[1] = h->g.ny;
    hd.n_cells[2] = h->g.nz;
    hd.parity = h->parity;
    hd.a = h->g.a;
    hd.rc = h->g.rc;
    hd.delta2 = h->g.delta2;
    hd.mass = h->mass;
    hd.rcap = h->rcap;
    hd.n_atoms = h->n_atoms;
    hd.steps_done = h->steps_done;
    hd.state_bytes = sb;
    hd.tables_hash = tables_hash(h);
    hd.rho_valid = h->rho_valid && !h->pending_clear;  // densities of a finished pass
    hd.force_valid = h->force_valid && !h->pending_clear;
    HIPCHK(h, hipMemcpyAsync(&hd.cnt, h->sc.cnt, sizeof(Counters), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(hd.scal, h->sc.scal, sizeof(hd.scal), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync((char *)host_out + sizeof(CkptHeader), h->state_ptr, (size_t)sb, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::memcpy(host_out, &hd, sizeof(hd));
    return MISA_OK;
}

int misa_load_checkpoint(misa_lattice *h, const void *host_in, int64_t bytes) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (!h->state_bound) return fail(h, MISA_ESTATE, "no state buffer bound (misa_bind_state)");
    if (!h->tables_set) return fail(h, MISA_ESTATE, "no potential tables (misa_set_potential_tables)");
    if (!host_in || bytes < (int64_t)sizeof(CkptHeader)) return fail(h, MISA_EINVAL, "checkpoint too short");
    CkptHeader hd;
    std::memcpy(&hd, host_in, sizeof(hd));
    const int64_t sb = carve(h, nullptr, nullptr);
    if (std::memcmp(hd.magic, CKPT_MAGIC, 8) != 0) return fail(h, MISA_EINVAL, "not a checkpoint of this library");
    if (hd.precision != h->precision || hd.use_mlp != (int)h->use_mlp || hd.n_cells[0] != h->g.nx ||
        hd.n_cells[1] != h->g.ny || hd.n_cells[2] != h->g.nz || hd.a != h->g.a || hd.rc != h->g.rc ||
        hd.delta2 != h->g.delta2 || hd.mass != h->mass || hd.rcap != h->rcap || hd.state_bytes != sb)
        return fail(h, MISA_EINVAL, "checkpoint of another lattice (box, a, rc, delta, mass, capacity or precision)");
    if (bytes < (int64_t)sizeof(CkptHeader) + sb) return fail(h, MISA_EINVAL, "checkpoint too short");
    if (hd.tables_hash != tables_hash(h))
        return fail(h, MISA_EINVAL, "checkpoint taken with other potential tables");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(h->state_ptr, (const char *)host_in + sizeof(CkptHeader), (size_t)sb, hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->sc.cnt, &hd.cnt, sizeof(Counters), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->sc.scal, hd.scal, sizeof(hd.scal), hipMemcpyHostToDevice));
    // cell grid and near-run-away marks empty, as after any finished pass
    HIPCHK(h, hipMemset(h->sc.mark, 0, sizeof(uint32_t) * (size_t)h->sc.mark_nwords));
    HIPCHK(h, hipMemset(h->sc.cell_n, 0, sizeof(int32_t) * (size_t)h->sc.cs_nblk * CS_CHUNK));
    if (h->parity != hd.parity) swap_uv(h);
    drop_graph(h);
    h->n_atoms = hd.n_atoms;
    h->steps_done = hd.steps_done;
    h->state_set = true;
    h->rho_valid = hd.rho_valid != 0;
    h->force_valid = hd.force_valid != 0;
    h->pending_clear = false;
    return MISA_OK;
}

int misa_atom_count(const misa_lattice *h, int64_t *n_atoms) {
    if (!h || !n_atoms) return fail(nullptr, MISA_EINVAL, "null argument");
    *n_atoms = h->n_atoms;
    return MISA_OK;
}

int misa_get_state(misa_lattice *h, double *x, double *v, int where) {
    int rc = check_ready(h, false);
    if (rc) return rc;
    if (where != MISA_HOST && where != MISA_DEVICE) return fail(h, MISA_EINVAL, "bad memory kind");
    const int64_t n = h->n_atoms;
    if (n == 0 || (!x && !v)) return MISA_OK;
    if (where == MISA_DEVICE) {
        HIPCHK(h, launch_gather_state(h, x, v));
        return MISA_OK;
    }
    HIPCHK(h, ensure_staging(h, sizeof(double) * 6 * n));
    double *dx = h->staging, *dv = h->staging + 3 * n;
    HIPCHK(h, launch_gather_state(h, x ? dx : nullptr, v ? dv : nullptr));
    if (x) HIPCHK(h, hipMemcpyAsync(x, dx, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, h->stream));
    if (v) HIPCHK(h, hipMemcpyAsync(v, dv, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MISA_OK;
}

int misa_set_pair_schedule(misa_lattice *h, int schedule) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (schedule != MISA_PAIRS_GATHER && schedule != MISA_PAIRS_HALF)
        return fail(h, MISA_EINVAL, "schedule must be MISA_PAIRS_GATHER or MISA_PAIRS_HALF");
    if (schedule == MISA_PAIRS_HALF) {
        if (h->precision != MISA_FP32)
            return fail(h, MISA_EINVAL, "the half-stencil schedule serves the float32 table and learned forms only");
        if (!h->half_fits)
            return fail(h, MISA_EINVAL, "the half-stencil schedule needs every axis a multiple of 16 cells");
    }
    if (schedule != h->pair_schedule) {
        h->rho_valid = h->force_valid = false;
        drop_graph(h);
    }
    h->pair_schedule = schedule;
    return MISA_OK;
}

int misa_compute_rho(misa_lattice *h) {
    int rc = check_ready(h, true);
    if (rc) return rc;
    return do_rho(h);
}

int misa_compute_force(misa_lattice *h, double *energies_dev) {
    int rc = check_ready(h, true);
    if (rc) return rc;
    if (!h->rho_valid || !h->pending_clear)
        return fail(h, MISA_ESTATE, "misa_compute_force needs misa_compute_rho on the same state first");
    if ((rc = do_force(h, energies_dev != nullptr, energies_dev, false))) return rc;
    return finish_force(h);
}

int misa_step(misa_lattice *h, int64_t nsteps, double dt_max, double dx_max, misa_step_stats *stats) {
    int rc = check_ready(h, true);
    if (rc) return rc;
    if (nsteps < 0 || !(dt_max > 0) || !std::isfinite(dt_max) || !std::isfinite(dx_max))
        return fail(h, MISA_EINVAL, "nsteps >= 0 and dt_max > 0 required");
    if (!h->force_valid) {
        if ((rc = do_rho(h))) return rc;
        if ((rc = do_force(h, false, nullptr, false))) return rc;
        if ((rc = finish_force(h))) return rc;
    }
    const bool fused = fused_kick(h);
    {
        GroupTimer t(h, MISA_TIMER_OTHER);
        HIPCHK(h, launch_dt_update(h, dt_max, dx_max, true));
    }
    int64_t s = 0;
    if (h->use_graph && !h->timing && nsteps >= 2) {
        // every step but the last issues the same kernels with the same arguments (dt
        // lives on the device), but on alternating copies of u and v: replay the two
        // captured steps in turn
        for (; s < nsteps - 1; ++s) {
            const int par = h->parity;
            if (!h->graph_exec[par] || h->graph_dt[par] != dt_max || h->graph_dx[par] != dx_max) {
                if (h->graph_exec[par]) (void)hipGraphExecDestroy(h->graph_exec[par]);
                h->graph_exec[par] = nullptr;
                if ((rc = capture_step(h, fused, dt_max, dx_max))) return rc;
            }
            HIPCHK(h, hipGraphLaunch(h->graph_exec[par], h->stream));
            swap_uv(h);
        }
    }
    for (; s < nsteps; ++s)
        if ((rc = step_body(h, s == nsteps - 1, fused, dt_max, dx_max))) return rc;
    double scal[8];
    Counters c;
    HIPCHK(h, hipMemcpyAsync(&c, h->sc.cnt, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (c.overflow && nsteps > 0) {
        // The failing step was undone and every later step of the call left the state
        // where it was (dt = 0); the densities, forces and energies of the last of them
        // belong to that state.  Take the step length of the state and clear the flag.
        h->steps_done += c.fail_step;
        HIPCHK(h, launch_dt_update(h, dt_max, dx_max, true));
    } else {
        h->steps_done += nsteps;
    }
    if (stats) {
        HIPCHK(h, hipMemcpyAsync(scal, h->sc.scal, sizeof(scal), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        std::memset(stats, 0, sizeof(*stats));
        stats->dt_next = scal[0];
        stats->time = scal[1];
        stats->vmax = scal[2];
        stats->e_kin = scal[3];
        stats->e_emb = nsteps > 0 ? scal[4] : 0.0;
        stats->e_pair = nsteps > 0 ? scal[5] : 0.0;
        stats->steps = h->steps_done;
        stats->n_runaway = c.n_run;
        stats->range_violations = c.range_viol;
        stats->overflow = c.overflow ? 1 : 0;
        stats->failed_step = c.overflow ? c.fail_step : -1;
        stats->dt = scal[6];
    }
    if (c.overflow && nsteps > 0)
        return fail(h, MISA_EOVERFLOW, "run-away capacity exceeded at step " + std::to_string(c.fail_step) +
                                           " of the call; the state is left at the start of that step");
    return MISA_OK;
}

// ---------------------------------------------------------------------------
// Batched replicas

}  // extern "C"

struct misa_batch {
    hipStream_t stream = nullptr;
    std::vector<misa_lattice *> box;
    std::string err;
    // box tables, two sets of n_boxes: set 0 with each box's current copy of u and v,
    // set 1 with the copies swapped; a step starts on one set and its kick-drift
    // hands over to the other
    std::vector<BoxRef> ref;
    std::vector<BoxPass> pass;
    std::vector<int2> items;
    BoxRef *d_ref = nullptr;
    BoxPass *d_pass = nullptr;
    int2 *d_items = nullptr;
    int32_t *d_off = nullptr;  // 3 (boxes + 1): offsets of the run-away work lists
    int64_t cap_boxes = 0, cap_items = 0;
    std::vector<int32_t> shape;                  // tile shape of each box (index into TILE_SHAPES)
    StencilEntry<float> *d_st = nullptr;         // [N_TILE_SHAPES][2][KMAX]: stencil per tile shape
    // graph of one regular batched step (misa_batch_set_graph), valid for graph_key
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};  // a step starting on table set 0 / 1
    std::vector<uint64_t> graph_key;
};

namespace {

int bfail(misa_batch *b, int code, const std::string &msg) {
    if (b)
        b->err = msg;
    else
        g_create_error = msg;
    return code;
}

#define BCHK(b, expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bfail((b), MISA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

// Box tables and the (box, tile) work list of the persistent passes, in box order.
int batch_tables(misa_batch *b) {
    const int nb = (int)b->box.size();
    b->ref.resize(2 * nb);
    b->pass.resize(2 * nb);
    b->items.clear();
    for (int k = 0; k < nb; ++k) {
        misa_lattice *h = b->box[k];
        const int sh = b->shape[k];
        Geom g = h->g;  // the box with the batch's tiling for it
        for (int a = 0; a < 3; ++a) {
            g.tshape[a] = TILE_SHAPES[sh][a];
            const uint32_t side = (uint32_t)(g.tshape[a] + 2 * HALO);
            g.tdiv[a] = (uint32_t)((0x100000000ull + side - 1) / side);
        }
        g.nt2[0] = (g.nx + g.tshape[0] - 1) / g.tshape[0];
        g.nt2[1] = (g.ny + g.tshape[1] - 1) / g.tshape[1];
        g.nt2[2] = (g.nz + g.tshape[2] - 1) / g.tshape[2];
        g.ntiles2 = g.nt2[0] * g.nt2[1] * g.nt2[2];
        g.ntiles2_pad = (g.ntiles2 + 7) / 8 * 8;
        b->ref[k] = BoxRef{h->S, h->sc, g, h->rcap, h->alt};
        b->pass[k] = BoxPass{g, pass_ptrs(h), sh, 0};
        swap_uv(h);
        b->ref[nb + k] = BoxRef{h->S, h->sc, g, h->rcap, h->alt};
        b->pass[nb + k] = BoxPass{g, pass_ptrs(h), sh, 0};
        swap_uv(h);
        for (int t = 0; t < g.ntiles2; ++t) b->items.push_back(int2{k, t});
    }
    if (nb > b->cap_boxes) {
        (void)hipFree(b->d_ref);
        (void)hipFree(b->d_pass);
        (void)hipFree(b->d_off);
        b->d_ref = nullptr;
        b->d_pass = nullptr;
        b->d_off = nullptr;
        b->cap_boxes = 0;
        BCHK(b, hipMalloc((void **)&b->d_ref, sizeof(BoxRef) * 2 * nb));
        BCHK(b, hipMalloc((void **)&b->d_pass, sizeof(BoxPass) * 2 * nb));
        BCHK(b, hipMalloc((void **)&b->d_off, sizeof(int32_t) * 3 * (nb + 1)));
        b->cap_boxes = nb;
    }

    if ((int64_t)b->items.size() > b->cap_items) {
        (void)hipFree(b->d_items);
        b->d_items = nullptr;
        b->cap_items = 0;
        BCHK(b, hipMalloc((void **)&b->d_items, sizeof(int2) * b->items.size()));
        b->cap_items = (int64_t)b->items.size();
    }
    BCHK(b, hipMemcpyAsync(b->d_ref, b->ref.data(), sizeof(BoxRef) * 2 * nb, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipMemcpyAsync(b->d_pass, b->pass.data(), sizeof(BoxPass) * 2 * nb, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipMemcpyAsync(b->d_items, b->items.data(), sizeof(int2) * b->items.size(), hipMemcpyHostToDevice,
                           b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));  // the host tables may change on the next call
    return MISA_OK;
}

}  // namespace

extern "C" {

int misa_batch_create(const misa_lattice_desc *descs, int32_t n_boxes, void *hip_stream, misa_batch **out) {
    if (!descs || !out || n_boxes < 1) return bfail(nullptr, MISA_EINVAL, "need descriptors, n_boxes >= 1 and out");
    if (n_boxes > BATCH_MAX_BOXES)
        return bfail(nullptr, MISA_EINVAL, "at most " + std::to_string(BATCH_MAX_BOXES) + " boxes per batch");
    *out = nullptr;
    const misa_lattice_desc &d0 = descs[0];
    for (int k = 0; k < n_boxes; ++k) {
        const misa_lattice_desc &d = descs[k];
        if (d.pair_precision != MISA_FP32)
            return bfail(nullptr, MISA_EINVAL, "batched boxes use pair_precision MISA_FP32");
        if (d.a != d0.a || d.rc != d0.rc || d.delta != d0.delta || d.mass != d0.mass)
            return bfail(nullptr, MISA_EINVAL, "batched boxes share a, rc, delta and mass (one stencil, one potential)");
    }
    misa_batch *b = new (std::nothrow) misa_batch();
    if (!b) return bfail(nullptr, MISA_ENOMEM, "host allocation failed");
    b->stream = (hipStream_t)hip_stream;
    for (int k = 0; k < n_boxes; ++k) {
        misa_lattice *h = nullptr;
        const int rc = misa_create_lattice(&descs[k], hip_stream, &h);
        if (rc) {
            const std::string m = "box " + std::to_string(k) + ": " + g_create_error;
            misa_batch_destroy(b);
            return bfail(nullptr, rc, m);
        }
        b->box.push_back(h);
    }
    {
        // the run-away passes index one list over all boxes with 32-bit integers
        int64_t run = 0, aff = 0;
        for (const misa_lattice *h : b->box) {
            run += h->rcap;
            aff += h->sc.affected_cap;
        }
        if (run >= INT32_MAX || aff >= INT32_MAX) {
            misa_batch_destroy(b);
            return bfail(nullptr, MISA_EINVAL, "run-away capacities of the batch sum beyond 2^31 - 1");
        }
    }
    b->shape.assign(n_boxes, 0);
    // The boxes share one stencil: its LDS offsets for every tile shape, from box 0.
    {
        const misa_lattice *h0 = b->box[0];
        std::vector<StencilEntry<float>> sts((size_t)N_TILE_SHAPES * 2 * KMAX, StencilEntry<float>{0, 0.f, 0.f, 0.f});
        for (int sh = 0; sh < N_TILE_SHAPES; ++sh) {
            const int px = TILE_SHAPES[sh][0] + 2 * HALO, py = TILE_SHAPES[sh][1] + 2 * HALO,
                      pz = TILE_SHAPES[sh][2] + 2 * HALO;
            for (int p = 0; p < 2; ++p)
                for (int k = 0; k < h0->K; ++k) {
                    const int64_t *c = &h0->stencil_canon[(p * h0->K + k) * 3];
                    const int pn = (int)(((p + c[0]) % 2 + 2) % 2);
                    const int dcx = (int)((p + c[0] - pn) / 2), dcy = (int)c[1], dcz = (int)c[2];
                    const int lds = (pn - p) * pz * py * px + (dcz * py + dcy) * px + dcx;
                    const double a = h0->g.a;
                    sts[((size_t)sh * 2 + p) * KMAX + k] =
                        StencilEntry<float>{lds, (float)(c[0] * 0.5 * a), (float)((c[1] + 0.5 * pn - 0.5 * p) * a),
                                            (float)((c[2] + 0.5 * pn - 0.5 * p) * a)};
                }
        }
        hipError_t e = hipMalloc((void **)&b->d_st, sizeof(StencilEntry<float>) * sts.size());
        if (e == hipSuccess)
            e = hipMemcpy(b->d_st, sts.data(), sizeof(StencilEntry<float>) * sts.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            const std::string m = std::string("stencil upload: ") + hipGetErrorString(e);
            misa_batch_destroy(b);
            return bfail(nullptr, MISA_EHIP, m);
        }
    }
    *out = b;
    return MISA_OK;
}

int misa_batch_destroy(misa_batch *b) {
    if (!b) return MISA_OK;
    for (misa_lattice *h : b->box) misa_destroy_lattice(h);
    (void)hipFree(b->d_ref);
    (void)hipFree(b->d_pass);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_off);
    (void)hipFree(b->d_st);
    for (hipGraphExec_t g : b->graph_exec)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return MISA_OK;
}

const char *misa_batch_last_error(const misa_batch *b) { return b ? b->err.c_str() : g_create_error.c_str(); }

int misa_batch_box(misa_batch *b, int32_t k, misa_lattice **out) {
    if (!b || !out) return bfail(b, MISA_EINVAL, "null argument");
    if (k < 0 || k >= (int32_t)b->box.size()) return bfail(b, MISA_EINVAL, "box index out of range");
    *out = b->box[k];
    return MISA_OK;
}

int misa_batch_set_potential_tables(misa_batch *b, const misa_table *f, const misa_table *phi,
                                    const misa_table *emb) {
    if (!b) return MISA_EINVAL;
    for (size_t k = 0; k < b->box.size(); ++k) {
        const int rc = misa_set_potential_tables(b->box[k], f, phi, emb);
        if (rc) return bfail(b, rc, "box " + std::to_string(k) + ": " + b->box[k]->err);
    }
    return MISA_OK;
}

int misa_batch_step(misa_batch *b, int64_t nsteps, double dt_max, double dx_max, misa_step_stats *stats) {
    if (!b) return MISA_EINVAL;
    if (nsteps < 0 || !(dt_max > 0) || !std::isfinite(dt_max) || !std::isfinite(dx_max))
        return bfail(b, MISA_EINVAL, "nsteps >= 0 and dt_max > 0 required");
    const int nb = (int)b->box.size();
    misa_lattice *h0 = b->box[0];
    int64_t max_sites = 0;
    int max_mark = 1, max_cells = 1;
    for (int k = 0; k < nb; ++k) {
        misa_lattice *h = b->box[k];
        int rc = check_ready(h, true);
        if (rc) return bfail(b, rc, "box " + std::to_string(k) + ": " + h->err);
        if (!lds_path(h))
            return bfail(b, MISA_EINVAL, "box " + std::to_string(k) + ": the persistent float32 passes are not usable");
        if (h->pair_schedule != MISA_PAIRS_GATHER)
            return bfail(b, MISA_EINVAL, "box " + std::to_string(k) + ": batched replicas use the gather schedule");
        // the same stencil and tables serve every box
        if (h->lds32.nwin != h0->lds32.nwin || h->lds32.k0 != h0->lds32.k0 || h->K != h0->K)
            return bfail(b, MISA_EINVAL, "boxes differ in tables or stencil");
        if (!h->force_valid) {
            if ((rc = do_rho(h)) || (rc = do_force(h, false, nullptr, false)) || (rc = finish_force(h)))
                return bfail(b, rc, "box " + std::to_string(k) + ": " + h->err);
        }
        if (h->pending_clear) {
            if ((rc = finish_force(h))) return bfail(b, rc, h->err);
        }
        if ((rc = [&] { HIPCHK(h, launch_dt_update(h, dt_max, dx_max, true)); return MISA_OK; }()))
            return bfail(b, rc, h->err);
        max_sites = std::max<int64_t>(max_sites, h->g.nsites);
        max_mark = std::max(max_mark, (int)h->sc.mark_nblk);
        max_cells = std::max(max_cells, (int)h->sc.cs_nblk);
    }
    int rc = batch_tables(b);
    if (rc) return rc;
    const int gx_sites = (int)std::min<int64_t>((max_sites + 255) / 256, 512);
    const int gx_small = 16;
    const double kf = ACC_UNIT / h0->mass;
    const hipStream_t st = b->stream;
    const int nitems = (int)b->items.size();
    const bool any_shape = std::any_of(b->shape.begin(), b->shape.end(), [](int32_t x) { return x != 0; });
    // One batched step on stream sq (box 0's stream field follows it, since the
    // persistent passes launch on h0->stream).  Kernel timing of the batch, when
    // enabled, accumulates on box 0's timers.
    // set: the table set the step starts on; after the kick-drift every kernel reads the other
    auto step_body = [&](bool last, hipStream_t sq, int set) -> int {
        const hipStream_t st = sq;
        h0->stream = sq;
        const BoxRef *ref0 = b->d_ref + (int64_t)set * nb, *ref = b->d_ref + (int64_t)(set ^ 1) * nb;
        const BoxPass *pass = b->d_pass + (int64_t)(set ^ 1) * nb;
        {
            GroupTimer t(h0, MISA_TIMER_KICK);
            BCHK(b, launchb_kick_drift(st, ref0, ref, nb, gx_sites, gx_small, kf));
        }
        {
            GroupTimer t(h0, MISA_TIMER_RUNAWAY);
            BCHK(b, launchb_rehash(st, ref, nb, gx_small));
            BCHK(b, launchb_runaway_build(st, ref, nb, gx_small, max_cells));
        }
        {
            GroupTimer t(h0, MISA_TIMER_RHO);
            BCHK(b, launch_rho_lds_batch(h0, pass, b->d_items, nitems, b->d_st, any_shape));
        }
        {
            GroupTimer t(h0, MISA_TIMER_RUNAWAY);
            BCHK(b, launchb_runaway_rho(h0, ref, nb, max_mark, b->d_off));
        }
        {
            GroupTimer t(h0, MISA_TIMER_FORCE);
            BCHK(b, launch_force_lds_batch(h0, pass, b->d_items, nitems, last, true, b->d_st, any_shape));
        }
        {
            GroupTimer t(h0, MISA_TIMER_RUNAWAY);
            BCHK(b, launchb_runaway_force(h0, ref, nb, last, b->d_off));
        }
        {
            GroupTimer t(h0, MISA_TIMER_OTHER);
            if (last) BCHK(b, launchb_energy_reduce(st, ref, nb));
        }
        {
            GroupTimer t(h0, MISA_TIMER_KICK);
            BCHK(b, launchb_final_kick_runaway(st, ref, nb, gx_small, kf));
        }
        {
            GroupTimer t(h0, MISA_TIMER_OTHER);
            BCHK(b, launchb_dt_update(st, ref, nb, h0->mass, dt_max, dx_max));
        }
        {
            GroupTimer t(h0, MISA_TIMER_RUNAWAY);
            BCHK(b, launchb_runaway_clear(st, ref, nb));
        }
        if (h0->timed.size() > 50000) BCHK(b, fold_timing(h0));
        h0->stream = b->stream;
        return MISA_OK;
    };
    int64_t s = 0;
    if (b->use_graph && !h0->timing && nsteps >= 2) {
        // the key: everything the captured launches bake in
        std::vector<uint64_t> key = {(uint64_t)nitems, (uint64_t)any_shape, (uint64_t)gx_sites, (uint64_t)max_mark,
                                     (uint64_t)max_cells,
                                     (uint64_t)(uintptr_t)b->d_ref, (uint64_t)(uintptr_t)b->d_pass,
                                     (uint64_t)(uintptr_t)b->d_items, (uint64_t)(uintptr_t)b->d_off};
        uint64_t bits;
        std::memcpy(&bits, &dt_max, 8);
        key.push_back(bits);
        std::memcpy(&bits, &dx_max, 8);
        key.push_back(bits);
        for (misa_lattice *h : b->box) key.push_back(h->gen);
        if (!b->graph_exec[0] || !b->graph_exec[1] || key != b->graph_key) {
            BCHK(b, hipStreamSynchronize(b->stream));
            for (int set = 0; set < 2; ++set) {
                if (b->graph_exec[set]) (void)hipGraphExecDestroy(b->graph_exec[set]);
                b->graph_exec[set] = nullptr;
                hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
                int brc = MISA_OK;
                if (e == hipSuccess) brc = step_body(false, b->cap_stream, set);
                h0->stream = b->stream;
                hipGraph_t graph = nullptr;
                const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(b->cap_stream, &graph) : e;
                if (brc) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return brc;
                }
                BCHK(b, e2);
                e = hipGraphInstantiate(&b->graph_exec[set], graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) b->graph_exec[set] = nullptr;
                BCHK(b, e);
            }
            b->graph_key = key;
        }
        for (; s < nsteps - 1; ++s) BCHK(b, hipGraphLaunch(b->graph_exec[s & 1], b->stream));
    }
    for (; s < nsteps; ++s)
        if ((rc = step_body(s == nsteps - 1, b->stream, (int)(s & 1)))) return rc;
    std::vector<double> scal(8 * (size_t)nb);
    std::vector<Counters> cnt(nb);
    for (int k = 0; k < nb; ++k) {
        misa_lattice *h = b->box[k];
        if (nsteps & 1) swap_uv(h);  // the host view follows the copy the last step wrote
        h->rho_valid = h->force_valid = true;
        h->pending_clear = false;
        BCHK(b, hipMemcpyAsync(&cnt[k], h->sc.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st));
    }
    BCHK(b, hipStreamSynchronize(st));
    int worst = MISA_OK;
    for (int k = 0; k < nb; ++k) {
        misa_lattice *h = b->box[k];
        if (cnt[k].overflow && nsteps > 0) {  // box k stopped at the start of its failing step
            h->steps_done += cnt[k].fail_step;
            BCHK(b, launch_dt_update(h, dt_max, dx_max, true));
            worst = bfail(b, MISA_EOVERFLOW, "box " + std::to_string(k) + ": run-away capacity exceeded at step " +
                                                 std::to_string(cnt[k].fail_step) +
                                                 " of the call; the box is left at the start of that step");
        } else {
            h->steps_done += nsteps;
        }
        if (stats) BCHK(b, hipMemcpyAsync(&scal[8 * k], h->sc.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    BCHK(b, hipStreamSynchronize(st));
    if (!stats) return worst;
    for (int k = 0; k < nb; ++k) {
        misa_step_stats &o = stats[k];
        const double *sc = &scal[8 * k];
        std::memset(&o, 0, sizeof(o));
        o.dt_next = sc[0];
        o.time = sc[1];
        o.vmax = sc[2];
        o.e_kin = sc[3];
        o.e_emb = nsteps > 0 ? sc[4] : 0.0;
        o.e_pair = nsteps > 0 ? sc[5] : 0.0;
        o.steps = b->box[k]->steps_done;
        o.n_runaway = cnt[k].n_run;
        o.range_violations = cnt[k].range_viol;
        o.overflow = cnt[k].overflow ? 1 : 0;
        o.failed_step = cnt[k].overflow ? cnt[k].fail_step : -1;
        o.dt = sc[6];
    }
    return worst;
}

int misa_batch_set_graph(misa_batch *b, int enable) {
    if (!b) return MISA_EINVAL;
    if (enable && !b->cap_stream) BCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    if (!enable)
        for (hipGraphExec_t &g : b->graph_exec) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    b->use_graph = enable != 0;
    return MISA_OK;
}

int misa_batch_set_tile_shape(misa_batch *b, int32_t k, int32_t shape) {
    if (!b) return MISA_EINVAL;
    if (k < 0 || k >= (int32_t)b->box.size()) return bfail(b, MISA_EINVAL, "box index out of range");
    if (shape < 0 || shape >= N_TILE_SHAPES) return bfail(b, MISA_EINVAL, "unknown tile shape");
    b->shape[k] = shape;
    return MISA_OK;
}

int misa_batch_get_tile_shape(misa_batch *b, int32_t k, int32_t *shape) {
    if (!b || !shape) return MISA_EINVAL;
    if (k < 0 || k >= (int32_t)b->box.size()) return bfail(b, MISA_EINVAL, "box index out of range");
    *shape = b->shape[k];
    return MISA_OK;
}

int misa_batch_autotune(misa_batch *b, int64_t probe_steps, double dt_max, double dx_max, int32_t *policy,
                        double *ms_per_step, int64_t *steps_done) {
    if (!b) return MISA_EINVAL;
    if (probe_steps < 1) return bfail(b, MISA_EINVAL, "probe_steps >= 1 required");
    const int nb = (int)b->box.size();
    // policy 0: every box on 8 x 8 x 8 tiles; policy 1: every box on the shape that
    // covers it with the fewest cells (8 x 8 x 8 on ties)
    std::vector<int32_t> cand[2];
    cand[0].assign(nb, 0);
    cand[1].assign(nb, 0);
    for (int k = 0; k < nb; ++k) {
        const Geom &g = b->box[k]->g;
        int64_t best = -1;
        for (int sh = 0; sh < N_TILE_SHAPES; ++sh) {
            const int *t = TILE_SHAPES[sh];
            const int64_t cells = (int64_t)((g.nx + t[0] - 1) / t[0] * t[0]) * ((g.ny + t[1] - 1) / t[1] * t[1]) *
                                  ((g.nz + t[2] - 1) / t[2] * t[2]);
            if (best < 0 || cells < best) {
                best = cells;
                cand[1][k] = sh;
            }
        }
    }
    const int npol = cand[1] == cand[0] ? 1 : 2;
    const std::vector<int32_t> before = b->shape;
    double ms[2] = {0.0, 0.0};
    int64_t done = 0;
    for (int pol = 0; pol < npol; ++pol) {
        b->shape = cand[pol];
        int rc = misa_batch_step(b, 1, dt_max, dx_max, nullptr);  // untimed: first launches of this tiling
        if (!rc) ++done;
        const auto t0 = std::chrono::steady_clock::now();
        if (!rc) rc = misa_batch_step(b, probe_steps, dt_max, dx_max, nullptr);  // synchronises at the end
        if (rc) {  // the tiling in force when the call began; *steps_done: the steps the boxes did advance
            b->shape = before;
            if (steps_done) *steps_done = done;
            return rc;
        }
        ms[pol] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
                  (double)probe_steps;
        done += probe_steps;
    }
    const int best = (npol == 2 && ms[1] < ms[0]) ? 1 : 0;
    b->shape = cand[best];
    if (policy) *policy = best;
    if (ms_per_step) {
        ms_per_step[0] = ms[0];
        ms_per_step[1] = npol == 2 ? ms[1] : ms[0];
    }
    if (steps_done) *steps_done = done;
    return MISA_OK;
}

int misa_defects(misa_lattice *h, int64_t *counts) {
    int rc = check_ready(h, false);
    if (rc) return rc;
    if (!counts) return fail(h, MISA_EINVAL, "null output");
    HIPCHK(h, ensure_staging(h, 3 * sizeof(unsigned long long)));
    unsigned long long *d = (unsigned long long *)h->staging;
    HIPCHK(h, hipMemsetAsync(d, 0, 3 * sizeof(unsigned long long), h->stream));
    HIPCHK(h, launch_defects(h, d));
    unsigned long long c[3];
    int32_t n_run = 0;
    HIPCHK(h, hipMemcpyAsync(c, d, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&n_run, &h->sc.cnt->n_run, sizeof(n_run), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    counts[0] = (int64_t)(c[0] - c[2]);
    counts[1] = (int64_t)c[1];
    counts[2] = n_run;
    counts[3] = (int64_t)c[0];
    return MISA_OK;
}

int misa_set_graph(misa_lattice *h, int enable) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (enable && !h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    if (!enable) drop_graph(h);
    h->use_graph = enable != 0;
    return MISA_OK;
}

int misa_set_timing(misa_lattice *h, int enable) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    HIPCHK(h, fold_timing(h));
    for (int k = 0; k < MISA_TIMER_COUNT; ++k) {
        h->timer_ms[k] = 0.0;
        h->timer_n[k] = 0;
    }
    h->timing = enable != 0;
    return MISA_OK;
}

int misa_get_timing(misa_lattice *h, misa_timing *out) {
    if (!h || !out) return fail(h, MISA_EINVAL, "null argument");
    HIPCHK(h, fold_timing(h));
    for (int k = 0; k < MISA_TIMER_COUNT; ++k) {
        out->ms[k] = h->timer_ms[k];
        out->launches[k] = h->timer_n[k];
    }
    return MISA_OK;
}

int misa_get_atom_field(misa_lattice *h, int field, double *out, int where) {
    int rc = check_ready(h, false);
    if (rc) return rc;
    if (field < MISA_FIELD_RHO || field > MISA_FIELD_FORCE) return fail(h, MISA_EINVAL, "unknown field");
    if (where != MISA_HOST && where != MISA_DEVICE) return fail(h, MISA_EINVAL, "bad memory kind");
    if (!out) return fail(h, MISA_EINVAL, "null output");
    const int64_t n = h->n_atoms * (field == MISA_FIELD_FORCE ? 3 : 1);
    if (n == 0) return MISA_OK;
    if (where == MISA_DEVICE) {
        HIPCHK(h, launch_gather_field(h, field, out));
        return MISA_OK;
    }
    HIPCHK(h, ensure_staging(h, sizeof(double) * n));
    HIPCHK(h, launch_gather_field(h, field, h->staging));
    HIPCHK(h, hipMemcpyAsync(out, h->staging, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return MISA_OK;
}

int64_t misa_debug_export(misa_lattice *h, int what, int64_t *host_out, int64_t capacity) {
    if (!h) return fail(nullptr, MISA_EINVAL, "null handle");
    if (what == MISA_EXPORT_STENCIL) {
        const int64_t need = (int64_t)h->stencil_canon.size();
        if (host_out) std::memcpy(host_out, h->stencil_canon.data(), sizeof(int64_t) * std::min(need, capacity));
        return h->K;
    }
    if (what == MISA_EXPORT_SLOTS) {
        int rc = check_ready(h, false);
        if (rc) return rc;
        const int64_t n = h->n_atoms;
        if (n == 0 || !host_out) return n;
        if (capacity < n) return fail(h, MISA_EINVAL, "capacity smaller than the atom count");
        HIPCHK(h, ensure_staging(h, sizeof(int64_t) * n));
        HIPCHK(h, launch_gather_slots(h, (int64_t *)h->staging));
        HIPCHK(h, hipMemcpyAsync(host_out, h->staging, sizeof(int64_t) * n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return n;
    }
    if (what == MISA_EXPORT_NEIGHBOURS) {
        int rc = check_ready(h, true);
        if (rc) return rc;
        if (h->use_mlp) return fail(h, MISA_EINVAL, "neighbour counts: table forms only (the learned form's f is a network)");
        const int64_t n = h->n_atoms;
        if (n == 0 || !host_out) return n;
        if (capacity < n) return fail(h, MISA_EINVAL, "capacity smaller than the atom count");
        // The density pass of the handle's own form with f = 1 inside rc counts every
        // pair it takes, run-away pairs included.  Afterwards the tables and counters
        // are restored and, if they were valid, the densities and F' recomputed (the
        // forces are not touched).
        const bool rho_was = h->rho_valid, force_was = h->force_valid;
        Counters c0;
        HIPCHK(h, hipMemcpyAsync(&c0, h->sc.cnt, sizeof(c0), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        const std::vector<double> ones(h->tab_y[0].size(), 1.0);
        misa_table unit = h->tab[0];
        unit.y = ones.data();
        rc = set_tables_impl(h, &unit, &h->tab[1], &h->tab[2]);
        if (!rc) rc = do_rho(h);
        std::vector<double> cnt(rc ? 0 : n);
        if (!rc) {
            HIPCHK(h, ensure_staging(h, sizeof(double) * n));
            HIPCHK(h, launch_gather_field(h, MISA_FIELD_RHO, h->staging));
            HIPCHK(h, hipMemcpyAsync(cnt.data(), h->staging, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
        }
        const int rc2 = set_tables_impl(h, &h->tab[0], &h->tab[1], &h->tab[2]);
        if (rc) return rc;
        if (rc2) return rc2;
        HIPCHK(h, hipMemcpyAsync(h->sc.cnt, &c0, sizeof(c0), hipMemcpyHostToDevice, h->stream));
        if (rho_was) {
            if ((rc = do_rho(h))) return rc;
            h->force_valid = force_was;
            if (force_was && (rc = finish_force(h))) return rc;  // as after a force pass: marks cleared
        }
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int64_t i = 0; i < n; ++i) {
            host_out[i] = (int64_t)std::llround(cnt[i]);
            if ((double)host_out[i] != cnt[i]) return fail(h, MISA_EHIP, "neighbour count not integral");
        }
        return n;
    }
    return fail(h, MISA_EINVAL, "unknown export");
}

}  // extern "C"
