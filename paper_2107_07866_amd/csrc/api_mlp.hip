// C ABI of the learned form: attaching surrogate networks to a lattice handle,
// the spline tables as training targets, the GPU trainer (fit to table samples,
// force matching on data collected from a lattice state).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "misa_internal.h"

using namespace misa;

struct misa_mlp_trainer {
    hipStream_t stream = nullptr;
    std::string err;
    struct Net {
        double x_lo = 0, x_hi = 0, y_shift = 0, y_scale = 1;
        float *w = nullptr, *m = nullptr, *v = nullptr, *q = nullptr;  // master, Adam moments, bfloat16 copy
        uint16_t *w2b = nullptr;
        int64_t step = 0;
        bool set = false;
        const double *sx = nullptr, *sy = nullptr, *sdy = nullptr;  // registered fit samples
        int64_t sn = 0;
        double lam = 1.0;
    } net[3];
    float *part = nullptr;       // [part_cap][MLP_NP]
    int64_t part_cap = 0;
    double *grad = nullptr;      // [MLP_NP]
    double *loss_part = nullptr; // [loss_cap]
    int64_t loss_cap = 0;
    double *loss_hist = nullptr; // [hist_cap]
    int64_t hist_cap = 0;
    // force matching
    int32_t *envs = nullptr;
    double *fm_x = nullptr, *fm_cf = nullptr, *fm_cp = nullptr, *fm_zero = nullptr, *fm_loss = nullptr;
    int64_t fm_cap = 0;
    double *scalar = nullptr;
    int32_t *tickets = nullptr;  // [3] finished blocks of a fused fit iteration, zero between launches
};

namespace {

thread_local std::string g_trainer_error;

int tfail(misa_mlp_trainer *t, int code, const std::string &msg) {
    if (t)
        t->err = msg;
    else
        g_trainer_error = msg;
    return code;
}

int hfail(misa_lattice *h, int code, const std::string &msg) {
    h->err = msg;
    return code;
}

#define TCHK(t, expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return tfail((t), MISA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

#define HCHK(h, expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return hfail((h), MISA_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

template <typename T>
hipError_t grow(T **p, int64_t &cap, int64_t need) {
    if (need <= cap) return hipSuccess;
    (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(need, 1));
    if (e == hipSuccess) cap = need;
    return e;
}

bool is_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return (u & 0xffffu) == 0u && std::isfinite(x);
}

uint16_t bf16_of(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return (uint16_t)(u >> 16);
}

bool valid_range(const misa_mlp_net *n) {
    return std::isfinite(n->x_lo) && std::isfinite(n->x_hi) && n->x_lo < n->x_hi && std::isfinite(n->y_shift) &&
           std::isfinite(n->y_scale) && n->y_scale != 0.0;
}

MlpNet meta_of(double lo, double hi, double sh, double sc, const float *p) {
    MlpNet m;
    m.p = p;
    m.c = (float)(0.5 * (lo + hi));
    m.s = (float)(2.0 / (hi - lo));
    m.y_shift = (float)sh;
    m.y_scale = (float)sc;
    m.x_lo = (float)lo;
    m.x_hi = (float)hi;
    return m;
}

MlpNet trainer_net(const misa_mlp_trainer::Net &N, const float *p) {
    return meta_of(N.x_lo, N.x_hi, N.y_shift, N.y_scale, p);
}

// Spline tables of a lattice handle (float64) at given points.
__global__ void k_table_eval(Tables<double> T, int fn, const double *__restrict__ x, int64_t n,
                             double *__restrict__ y, double *__restrict__ dy) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double xi = x[i];
        const TabMeta<double> &m = fn == MISA_FN_EMB ? T.em : T.fm;
        if (fn == MISA_FN_EMB && xi > m.x_last) {
            y[i] = m.y_last + m.d_last * (xi - m.x_last);
            dy[i] = m.d_last;
            continue;
        }
        const double p = (xi - m.x0) * m.inv_h;
        int k = (int)p;
        k = k < m.nseg - 1 ? k : m.nseg - 1;
        k = k > 0 ? k : 0;
        const double t = p - (double)k;
        if (fn == MISA_FN_EMB) {
            const Q4<double> c = T.emb[2 * k], d = T.emb[2 * k + 1];
            y[i] = ((c.w * t + c.z) * t + c.y) * t + c.x;
            dy[i] = (d.z * t + d.y) * t + d.x;
        } else {
            const Q4<double> a = T.force[2 * k], b = T.force[2 * k + 1];
            const Q4<double> c = fn == MISA_FN_F ? T.f[k] : T.phi[k];
            y[i] = ((c.w * t + c.z) * t + c.y) * t + c.x;
            dy[i] = fn == MISA_FN_F ? (a.z * t + a.y) * t + a.x : (b.y * t + b.x) * t + a.w;
        }
    }
}

// Force-matching data: one thread per requested site, float64 pair geometry.
template <typename Real>
__global__ void k_collect(State S, Geom g, Tables<double> T, const int32_t *__restrict__ canon, int K,
                          const int64_t *__restrict__ sites, int64_t n, double *__restrict__ r_out,
                          double *__restrict__ dhat, double *__restrict__ fpj_out, double *__restrict__ fpi_out,
                          double *__restrict__ fref) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t s = sites[q];
    const int p = s >= g.ncell ? 1 : 0;
    const int64_t c = s - p * g.ncell;
    const int cx = (int)(c % g.nx), cy = (int)((c / g.nx) % g.ny), cz = (int)(c / ((int64_t)g.nx * g.ny));
    const int X = 2 * cx + p;
    const double ux = S.ux[s];
    const bool vac = ux > VACANT_TEST;
    const double ui[3] = {ux, S.uy[s], S.uz[s]};
    const double fi = vac ? 0.0 : (double)((const Real *)S.fp)[s];
    double F[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < MISA_FM_SLOTS; ++k) {
        const int64_t o = q * MISA_FM_SLOTS + k;
        r_out[o] = 0.0;
        dhat[3 * o] = dhat[3 * o + 1] = dhat[3 * o + 2] = 0.0;
        fpj_out[o] = 0.0;
        if (vac || k >= K) continue;
        const int dX = canon[(p * K + k) * 3], dY = canon[(p * K + k) * 3 + 1], dZ = canon[(p * K + k) * 3 + 2];
        const int X2 = X + dX, Y2 = cy + dY, Z2 = cz + dZ;
        const int p2 = X2 & 1;
        const int cx2 = (X2 - p2) / 2;  // X2 - p2 is even
        // site offset vector from lattice-id coordinates (Sec. 3): (X a / 2, (Y + (X & 1) / 2) a, ...)
        const double o3[3] = {0.5 * g.a * (double)dX, g.a * ((double)dY + 0.5 * (double)(p2 - p)),
                              g.a * ((double)dZ + 0.5 * (double)(p2 - p))};
        const int64_t sj = (int64_t)p2 * g.ncell +
                           ((int64_t)wrap_index(Z2, g.nz) * g.ny + wrap_index(Y2, g.ny)) * g.nx + wrap_index(cx2, g.nx);
        const double uxj = S.ux[sj];
        if (uxj > VACANT_TEST) continue;
        const double d[3] = {o3[0] + (uxj - ui[0]), o3[1] + (S.uy[sj] - ui[1]), o3[2] + (S.uz[sj] - ui[2])};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < g.rc2)) continue;
        const double r = sqrt(r2);
        const double fj = (double)((const Real *)S.fp)[sj];
        const double pp = (r - T.fm.x0) * T.fm.inv_h;
        int sg = (int)pp;
        sg = sg < T.fm.nseg - 1 ? sg : T.fm.nseg - 1;
        sg = sg > 0 ? sg : 0;
        const double t = pp - (double)sg;
        const Q4<double> a = T.force[2 * sg], b = T.force[2 * sg + 1];
        const double df = (a.z * t + a.y) * t + a.x, dph = (b.y * t + b.x) * t + a.w;
        const double sc = (fi + fj) * df + dph;
        r_out[o] = r;
        for (int e = 0; e < 3; ++e) {
            dhat[3 * o + e] = d[e] / r;
            F[e] += sc * d[e] / r;
        }
        fpj_out[o] = fj;
    }
    fpi_out[q] = fi;
    for (int e = 0; e < 3; ++e) fref[3 * q + e] = F[e];
}

int ensure_scratch(misa_mlp_trainer *t, int64_t blocks, int64_t losses, int64_t hist) {
    TCHK(t, grow(&t->part, t->part_cap, blocks * (int64_t)MLP_NP));
    TCHK(t, grow(&t->loss_part, t->loss_cap, losses));
    TCHK(t, grow(&t->loss_hist, t->hist_cap, hist));
    return MISA_OK;
}

double lr_at(const misa_fit_opts *o, int64_t i) {
    if (o->iters <= 1) return o->lr;
    const double c = 0.5 * (1.0 + std::cos(M_PI * (double)i / (double)(o->iters - 1)));
    return o->lr_final + (o->lr - o->lr_final) * c;
}

int check_opts(misa_mlp_trainer *t, const misa_fit_opts *o) {
    if (!o) return tfail(t, MISA_EINVAL, "null options");
    if (o->iters < 1 || o->batch < 1 || !(o->lr > 0) || !(o->lr_final >= 0) || !(o->lambda >= 0))
        return tfail(t, MISA_EINVAL, "options: iters >= 1, batch >= 1, lr > 0, lr_final >= 0, lambda >= 0");
    return MISA_OK;
}

// Sobolev-mode gradient job of network f over its registered samples.
GradJob fit_job(misa_mlp_trainer *t, int fn, const float *pw, int64_t batch, uint64_t seed, double *loss_part,
                float *part) {
    misa_mlp_trainer::Net &N = t->net[fn];
    GradJob J{};
    J.p = pw;
    const MlpNet m = trainer_net(N, pw);
    J.c = m.c;
    J.s = m.s;
    J.y_shift = m.y_shift;
    J.y_scale = m.y_scale;
    J.x = N.sx;
    J.n = N.sn;
    J.y = N.sy;
    J.dy = N.sdy;
    J.lam = (float)N.lam;
    J.seed = seed;
    J.step = (uint64_t)N.step;
    J.batch = batch;
    J.cval = J.cder = nullptr;
    J.part = part;
    J.loss_part = loss_part;
    return J;
}

}  // namespace

extern "C" {

int misa_set_mlp(misa_lattice *h, int fn, const misa_mlp_net *net) {
    if (!h) return MISA_EINVAL;
    if (!h->use_mlp) return hfail(h, MISA_ESTATE, "misa_set_mlp needs a handle created with pair_precision MISA_MLP");
    if (fn < 0 || fn > 2 || !net) return hfail(h, MISA_EINVAL, "fn must be MISA_FN_F, MISA_FN_PHI or MISA_FN_EMB");
    if (!valid_range(net)) return hfail(h, MISA_EINVAL, "network range or scaling invalid");
    for (int j = 0; j < MLP_NP; ++j)
        if (!is_bf16(net->params[j]))
            return hfail(h, MISA_EINVAL, "weight " + std::to_string(j) + " is not a bfloat16 value");
    std::vector<uint16_t> w2(MLP_H * MLP_H);
    for (int j = 0; j < MLP_H * MLP_H; ++j) w2[j] = bf16_of(net->params[OFF_W2 + j]);
    MlpAttached &A = h->mlp;
    if (!h->pairbuf) {  // f'(r) per pair, kept from the rho pass for the force pass (either schedule)
        const hipError_t e = hipMalloc((void **)&h->pairbuf, sizeof(float) * (size_t)h->K * (size_t)h->g.nsites);
        if (e != hipSuccess) {
            h->pairbuf = nullptr;
            return hfail(h, MISA_ENOMEM, std::string("pair buffer of the learned form: ") + hipGetErrorString(e));
        }
    }
    if (!A.p[fn]) HCHK(h, hipMalloc((void **)&A.p[fn], sizeof(float) * MLP_NP));
    if (!A.w2b[fn]) HCHK(h, hipMalloc((void **)&A.w2b[fn], sizeof(uint16_t) * MLP_H * MLP_H));
    HCHK(h, hipMemcpyAsync(A.p[fn], net->params, sizeof(float) * MLP_NP, hipMemcpyHostToDevice, h->stream));
    HCHK(h, hipMemcpyAsync(A.w2b[fn], w2.data(), sizeof(uint16_t) * w2.size(), hipMemcpyHostToDevice, h->stream));
    HCHK(h, hipStreamSynchronize(h->stream));
    A.net[fn] = meta_of(net->x_lo, net->x_hi, net->y_shift, net->y_scale, A.p[fn]);
    A.set[fn] = true;
    h->rho_valid = h->force_valid = false;
    misa::drop_graph(h);  // the networks' ranges are kernel arguments of the captured step
    return MISA_OK;
}

int misa_table_eval(misa_lattice *h, int fn, const double *x, int64_t n, double *y, double *dy) {
    if (!h) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || n < 0 || (n > 0 && (!x || !y || !dy)))
        return hfail(h, MISA_EINVAL, "bad function id or arrays");
    if (!h->tables_set) return hfail(h, MISA_ESTATE, "no potential tables (misa_set_potential_tables)");
    if (n == 0) return MISA_OK;
    Tables<double> T;
    T.f = h->t64.f;
    T.force = h->t64.force;
    T.phi = h->t64.phi;
    T.emb = h->t64.emb;
    T.fm = h->t64.fm;
    T.em = h->t64.em;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_table_eval, dim3(blocks), dim3(256), 0, h->stream, T, fn, x, n, y, dy);
    HCHK(h, hipGetLastError());
    return MISA_OK;
}

int misa_mlp_collect(misa_lattice *h, const int64_t *sites, int64_t n, double *r, double *dhat, double *fp_j,
                     double *fp_i, double *f_ref) {
    if (!h) return MISA_EINVAL;
    if (n < 0 || (n > 0 && (!sites || !r || !dhat || !fp_j || !fp_i || !f_ref)))
        return hfail(h, MISA_EINVAL, "bad arrays");
    if (!h->state_set || !h->tables_set || !h->rho_valid)
        return hfail(h, MISA_ESTATE, "misa_mlp_collect needs tables, a state and misa_compute_rho first");
    if (h->K > MISA_FM_SLOTS) return hfail(h, MISA_EINVAL, "stencil longer than MISA_FM_SLOTS");
    if (n == 0) return MISA_OK;
    std::vector<int64_t> st(n);
    const int64_t nid = 2 * h->g.ncell;
    for (int64_t i = 0; i < n; ++i) {
        if (sites[i] < 0 || sites[i] >= nid) return hfail(h, MISA_EINVAL, "lattice id out of range");
        st[i] = storage_of_lattice_id(sites[i], h->g);
    }
    std::vector<int32_t> canon(h->stencil_canon.begin(), h->stencil_canon.end());
    int64_t *d_sites = nullptr;
    int32_t *d_canon = nullptr;
    HCHK(h, hipMalloc((void **)&d_sites, sizeof(int64_t) * n));
    hipError_t e = hipMalloc((void **)&d_canon, sizeof(int32_t) * canon.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d_sites, st.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_canon, canon.data(), sizeof(int32_t) * canon.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        Tables<double> T;
        T.f = h->t64.f;
        T.force = h->t64.force;
        T.phi = h->t64.phi;
        T.emb = h->t64.emb;
        T.fm = h->t64.fm;
        T.em = h->t64.em;
        const int blocks = (int)((n + 127) / 128);
        if (h->precision == MISA_FP64)
            hipLaunchKernelGGL(k_collect<double>, dim3(blocks), dim3(128), 0, h->stream, h->S, h->g, T, d_canon, h->K,
                               d_sites, n, r, dhat, fp_j, fp_i, f_ref);
        else
            hipLaunchKernelGGL(k_collect<float>, dim3(blocks), dim3(128), 0, h->stream, h->S, h->g, T, d_canon, h->K,
                               d_sites, n, r, dhat, fp_j, fp_i, f_ref);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d_sites);
    (void)hipFree(d_canon);
    HCHK(h, e);
    return MISA_OK;
}

int misa_mlp_trainer_create(void *hip_stream, misa_mlp_trainer **out) {
    if (!out) return tfail(nullptr, MISA_EINVAL, "null output pointer");
    *out = nullptr;
    misa_mlp_trainer *t = new (std::nothrow) misa_mlp_trainer();
    if (!t) return tfail(nullptr, MISA_ENOMEM, "host allocation failed");
    t->stream = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc((void **)&t->grad, sizeof(double) * MLP_NP);
    if (e == hipSuccess) e = hipMalloc((void **)&t->scalar, sizeof(double) * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&t->tickets, sizeof(int32_t) * 3);
    if (e == hipSuccess) e = hipMemset(t->tickets, 0, sizeof(int32_t) * 3);
    for (int f = 0; f < 3 && e == hipSuccess; ++f) {
        auto &N = t->net[f];
        float **bufs[] = {&N.w, &N.m, &N.v, &N.q};
        for (float **b : bufs)
            if (e == hipSuccess) e = hipMalloc((void **)b, sizeof(float) * MLP_NP);
        if (e == hipSuccess) e = hipMalloc((void **)&N.w2b, sizeof(uint16_t) * MLP_H * MLP_H);
    }
    if (e != hipSuccess) {
        misa_mlp_trainer_destroy(t);
        return tfail(nullptr, MISA_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    *out = t;
    return MISA_OK;
}

int misa_mlp_trainer_destroy(misa_mlp_trainer *t) {
    if (!t) return MISA_OK;
    (void)hipStreamSynchronize(t->stream);
    void *ptrs[] = {t->part, t->grad, t->loss_part, t->loss_hist, t->envs, t->fm_x, t->fm_cf,
                    t->fm_cp, t->fm_zero, t->fm_loss, t->scalar, t->tickets};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &N : t->net) {
        void *q[] = {N.w, N.m, N.v, N.q, N.w2b};
        for (void *p : q)
            if (p) (void)hipFree(p);
    }
    delete t;
    return MISA_OK;
}

const char *misa_mlp_last_error(const misa_mlp_trainer *t) {
    return t ? t->err.c_str() : g_trainer_error.c_str();
}

int misa_mlp_trainer_set(misa_mlp_trainer *t, int fn, const misa_mlp_net *net) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || !net) return tfail(t, MISA_EINVAL, "bad function id");
    if (!valid_range(net)) return tfail(t, MISA_EINVAL, "network range or scaling invalid");
    for (int j = 0; j < MLP_NP; ++j)
        if (!std::isfinite(net->params[j])) return tfail(t, MISA_EINVAL, "non-finite weight");
    auto &N = t->net[fn];
    N.x_lo = net->x_lo;
    N.x_hi = net->x_hi;
    N.y_shift = net->y_shift;
    N.y_scale = net->y_scale;
    TCHK(t, hipMemcpyAsync(N.w, net->params, sizeof(float) * MLP_NP, hipMemcpyHostToDevice, t->stream));
    TCHK(t, hipMemsetAsync(N.m, 0, sizeof(float) * MLP_NP, t->stream));
    TCHK(t, hipMemsetAsync(N.v, 0, sizeof(float) * MLP_NP, t->stream));
    TCHK(t, launch_round_weights(t->stream, N.w, N.q, N.w2b));
    TCHK(t, hipStreamSynchronize(t->stream));
    N.step = 0;
    N.set = true;
    return MISA_OK;
}

int misa_mlp_trainer_get(misa_mlp_trainer *t, int fn, misa_mlp_net *net, float *master) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || !net) return tfail(t, MISA_EINVAL, "bad function id");
    auto &N = t->net[fn];
    if (!N.set) return tfail(t, MISA_ESTATE, "network not set (misa_mlp_trainer_set)");
    std::memset(net, 0, sizeof(*net));
    net->x_lo = N.x_lo;
    net->x_hi = N.x_hi;
    net->y_shift = N.y_shift;
    net->y_scale = N.y_scale;
    TCHK(t, hipMemcpyAsync(net->params, N.q, sizeof(float) * MLP_NP, hipMemcpyDeviceToHost, t->stream));
    if (master) TCHK(t, hipMemcpyAsync(master, N.w, sizeof(float) * MLP_NP, hipMemcpyDeviceToHost, t->stream));
    TCHK(t, hipStreamSynchronize(t->stream));
    return MISA_OK;
}

int misa_mlp_eval(misa_mlp_trainer *t, int fn, int path, const double *x, int64_t n, double *y, double *dy) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || (path != 0 && path != 1) || n < 0 || (n > 0 && (!x || !y || !dy)))
        return tfail(t, MISA_EINVAL, "bad arguments");
    auto &N = t->net[fn];
    if (!N.set) return tfail(t, MISA_ESTATE, "network not set (misa_mlp_trainer_set)");
    TCHK(t, launch_mlp_eval(t->stream, path, trainer_net(N, N.q), N.w2b, x, n, y, dy));
    return MISA_OK;
}

int misa_mlp_grad(misa_mlp_trainer *t, int fn, const double *x, const double *c_val, const double *c_der, int64_t n,
                  double *grad) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || n < 1 || !x || !c_val || !c_der || !grad) return tfail(t, MISA_EINVAL, "bad arguments");
    auto &N = t->net[fn];
    if (!N.set) return tfail(t, MISA_ESTATE, "network not set (misa_mlp_trainer_set)");
    const int64_t nblk = (n + GRAD_SAMPLES - 1) / GRAD_SAMPLES;
    if (nblk > (int64_t)1 << 20) return tfail(t, MISA_EINVAL, "too many samples for one call");
    int rc = ensure_scratch(t, nblk, 1, 1);
    if (rc) return rc;
    GradJob J{};
    const MlpNet m = trainer_net(N, N.q);
    J.p = N.q;
    J.c = m.c;
    J.s = m.s;
    J.y_shift = m.y_shift;
    J.y_scale = m.y_scale;
    J.x = x;
    J.n = n;
    J.cval = c_val;
    J.cder = c_der;
    J.part = t->part;
    J.loss_part = nullptr;
    TCHK(t, launch_grad(t->stream, J, (int)nblk));
    TCHK(t, launch_grad_sum(t->stream, t->part, (int)nblk, grad));
    return MISA_OK;
}

int misa_mlp_adam(misa_mlp_trainer *t, int fn, const double *grad, double lr) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || !grad || !(lr > 0)) return tfail(t, MISA_EINVAL, "bad arguments");
    auto &N = t->net[fn];
    if (!N.set) return tfail(t, MISA_ESTATE, "network not set (misa_mlp_trainer_set)");
    N.step += 1;
    TCHK(t, launch_adam(t->stream, N.w, N.m, N.v, grad, N.q, lr, N.step));
    TCHK(t, launch_round_weights(t->stream, N.w, N.q, N.w2b));
    return MISA_OK;
}

}  // extern "C"

namespace {
// Fit networks fns[0 .. nnet - 1] together: one launch of k_fit_step per iteration
// for all of them (each draws its own mini-batches, as when fitted alone, so the
// result does not depend on which networks share the launches).
// Network fns[k] draws with seed o->seed + seed_step fns[k].
int fit_fused(misa_mlp_trainer *t, int nnet, const int *fns, const double *const *x, const double *const *y,
              const double *const *dy, const int64_t *n, const misa_fit_opts *o, uint64_t seed_step,
              double *loss) {
    int rc = check_opts(t, o);
    if (rc) return rc;
    if (nnet < 1 || nnet > 3 || !fns || !x || !y || !dy || !n) return tfail(t, MISA_EINVAL, "bad arguments");
    for (int k = 0; k < nnet; ++k) {
        if (fns[k] < 0 || fns[k] > 2 || n[k] < 1 || !x[k] || !y[k] || !dy[k])
            return tfail(t, MISA_EINVAL, "bad arguments");
        for (int l = 0; l < k; ++l)
            if (fns[l] == fns[k]) return tfail(t, MISA_EINVAL, "a network listed twice");
        if (!t->net[fns[k]].set) return tfail(t, MISA_ESTATE, "network not set (misa_mlp_trainer_set)");
    }
    const int64_t nblk = (o->batch + GRAD_SAMPLES - 1) / GRAD_SAMPLES;
    if (nblk > 65535) return tfail(t, MISA_EINVAL, "batch too large");
    const int64_t tail = std::max<int64_t>(1, o->iters / 100);
    rc = ensure_scratch(t, nnet * nblk, nnet * nblk, nnet * tail);
    if (rc) return rc;
    for (int k = 0; k < nnet; ++k) {
        auto &N = t->net[fns[k]];
        N.sx = x[k];
        N.sy = y[k];
        N.sdy = dy[k];
        N.sn = n[k];
        N.lam = o->lambda;
    }
    for (int64_t i = 0; i < o->iters; ++i) {
        FitSteps F{};
        F.nnet = nnet;
        F.lr = lr_at(o, i);
        for (int k = 0; k < nnet; ++k) {
            auto &N = t->net[fns[k]];
            const float *pw = o->quantize ? N.q : N.w;
            FitStep &S = F.s[k];
            S.J = fit_job(t, fns[k], pw, o->batch, o->seed + seed_step * (uint64_t)fns[k], t->loss_part + k * nblk,
                          t->part + k * nblk * MLP_NP);
            N.step += 1;
            S.w = N.w;
            S.m = N.m;
            S.v = N.v;
            S.q = N.q;
            S.bc1 = 1.0 - std::pow(0.9, (double)N.step);
            S.bc2 = 1.0 - std::pow(0.999, (double)N.step);
            S.ticket = t->tickets + k;
            S.loss_hist = t->loss_hist + k * tail;
            S.slot = i >= o->iters - tail ? (int)(i - (o->iters - tail)) : -1;
        }
        TCHK(t, launch_fit_step(t->stream, F, (int)nblk));
    }
    for (int k = 0; k < nnet; ++k) {
        auto &N = t->net[fns[k]];
        TCHK(t, launch_round_weights(t->stream, N.w, N.q, N.w2b));
    }
    std::vector<double> h(nnet * tail);
    TCHK(t, hipMemcpyAsync(h.data(), t->loss_hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, t->stream));
    TCHK(t, hipStreamSynchronize(t->stream));
    if (loss)
        for (int k = 0; k < nnet; ++k) {
            double s = 0.0;
            for (int64_t j = 0; j < tail; ++j) s += h[k * tail + j];
            loss[k] = s / (double)tail / (double)o->batch;
        }
    return MISA_OK;
}
}  // namespace

extern "C" {

int misa_mlp_fit(misa_mlp_trainer *t, int fn, const double *x, const double *y, const double *dy, int64_t n,
                 const misa_fit_opts *o, double *loss) {
    if (!t) return MISA_EINVAL;
    if (fn < 0 || fn > 2 || n < 1 || !x || !y || !dy) return tfail(t, MISA_EINVAL, "bad arguments");
    return fit_fused(t, 1, &fn, &x, &y, &dy, &n, o, 0, loss);
}

int misa_mlp_fit_many(misa_mlp_trainer *t, int nnet, const int *fns, const double *const *x,
                      const double *const *y, const double *const *dy, const int64_t *n, const misa_fit_opts *o,
                      double *loss) {
    if (!t) return MISA_EINVAL;
    return fit_fused(t, nnet, fns, x, y, dy, n, o, 1, loss);
}

int misa_mlp_force_match(misa_mlp_trainer *t, const double *r, const double *dhat, const double *fp_j,
                         const double *fp_i, const double *f_ref, int64_t n_env, const misa_fit_opts *o,
                         double *loss) {
    if (!t) return MISA_EINVAL;
    if (n_env < 1 || !r || !dhat || !fp_j || !fp_i || !f_ref) return tfail(t, MISA_EINVAL, "bad arguments");
    int rc = check_opts(t, o);
    if (rc) return rc;
    for (int f = 0; f < 2; ++f)
        if (!t->net[f].set || !t->net[f].sx)
            return tfail(t, MISA_ESTATE, "force matching needs the f and phi networks set and fitted (misa_mlp_fit)");
    if (o->batch > n_env) return tfail(t, MISA_EINVAL, "batch larger than the number of sampled atoms");
    const int nb = o->batch;
    const int64_t npair = (int64_t)nb * MISA_FM_SLOTS;
    const int64_t nblk_fm = (npair + GRAD_SAMPLES - 1) / GRAD_SAMPLES;
    const int64_t sob_batch = 4096;
    const int64_t nblk_sob = sob_batch / GRAD_SAMPLES;
    if (nblk_fm + nblk_sob > 65535) return tfail(t, MISA_EINVAL, "batch too large");
    const int64_t tail = std::max<int64_t>(1, o->iters / 100);
    rc = ensure_scratch(t, 2 * (nblk_fm + nblk_sob), std::max<int64_t>(nb, nblk_sob), tail);
    if (rc) return rc;
    if (npair > t->fm_cap) {
        void *old[] = {t->envs, t->fm_x, t->fm_cf, t->fm_cp, t->fm_zero, t->fm_loss};
        for (void *p : old)
            if (p) (void)hipFree(p);
        t->envs = nullptr;
        t->fm_x = t->fm_cf = t->fm_cp = t->fm_zero = t->fm_loss = nullptr;
        t->fm_cap = 0;
        TCHK(t, hipMalloc((void **)&t->envs, sizeof(int32_t) * nb));
        TCHK(t, hipMalloc((void **)&t->fm_x, sizeof(double) * npair));
        TCHK(t, hipMalloc((void **)&t->fm_cf, sizeof(double) * npair));
        TCHK(t, hipMalloc((void **)&t->fm_cp, sizeof(double) * npair));
        TCHK(t, hipMalloc((void **)&t->fm_zero, sizeof(double) * npair));
        TCHK(t, hipMalloc((void **)&t->fm_loss, sizeof(double) * nb));
        TCHK(t, hipMemsetAsync(t->fm_zero, 0, sizeof(double) * npair, t->stream));
        t->fm_cap = npair;
    }
    TCHK(t, launch_fm_norm(t->stream, f_ref, n_env, t->scalar));
    double mean_f2 = 0.0;
    TCHK(t, hipMemcpyAsync(&mean_f2, t->scalar, sizeof(double), hipMemcpyDeviceToHost, t->stream));
    TCHK(t, hipStreamSynchronize(t->stream));
    if (!(mean_f2 > 0.0)) return tfail(t, MISA_EINVAL, "reference forces are all zero");
    for (int64_t i = 0; i < o->iters; ++i) {
        auto &Nf = t->net[0], &Np = t->net[1];
        const float *pf = o->quantize ? Nf.q : Nf.w;
        const float *pp = o->quantize ? Np.q : Np.w;
        FmJob F{};
        F.nf = trainer_net(Nf, pf);
        F.np = trainer_net(Np, pp);
        F.r = r;
        F.dhat = dhat;
        F.fpj = fp_j;
        F.fpi = fp_i;
        F.fref = f_ref;
        F.n_env = n_env;
        F.envs = t->envs;
        F.nb = nb;
        F.inv_norm = 1.0 / ((double)nb * mean_f2);
        F.x_out = t->fm_x;
        F.cf = t->fm_cf;
        F.cp = t->fm_cp;
        F.loss_part = t->fm_loss;
        TCHK(t, launch_fm(t->stream, F, o->seed, (uint64_t)i, t->envs));
        if (i >= o->iters - tail)
            TCHK(t, launch_sum_into(t->stream, t->fm_loss, nb, t->loss_hist, (int)(i - (o->iters - tail))));
        // both networks' gradients (force-matching pairs, then the Sobolev term on the
        // function's own samples), their sums and Adam steps: one launch
        FitSteps FS{};
        FS.nnet = 2;
        FS.lr = lr_at(o, i);
        for (int f = 0; f < 2; ++f) {
            auto &N = t->net[f];
            const float *pw = f == 0 ? pf : pp;
            float *part = t->part + (int64_t)f * (nblk_fm + nblk_sob) * MLP_NP;
            GradJob J{};
            const MlpNet m = trainer_net(N, pw);
            J.p = pw;
            J.c = m.c;
            J.s = m.s;
            J.y_shift = m.y_shift;
            J.y_scale = m.y_scale;
            J.x = t->fm_x;
            J.n = npair;
            J.cval = t->fm_zero;
            J.cder = f == 0 ? t->fm_cf : t->fm_cp;
            J.part = part;
            J.loss_part = nullptr;
            FitStep &S = FS.s[f];
            S.J = J;
            S.J2 = fit_job(t, f, pw, sob_batch, o->seed ^ 0x5eedull, nullptr, part + nblk_fm * MLP_NP);
            S.nblk1 = (int)nblk_fm;
            N.step += 1;
            S.w = N.w;
            S.m = N.m;
            S.v = N.v;
            S.q = N.q;
            S.bc1 = 1.0 - std::pow(0.9, (double)N.step);
            S.bc2 = 1.0 - std::pow(0.999, (double)N.step);
            S.ticket = t->tickets + f;
            S.loss_hist = nullptr;
            S.slot = -1;
        }
        TCHK(t, launch_fit_step(t->stream, FS, (int)(nblk_fm + nblk_sob)));
    }
    for (int f = 0; f < 2; ++f)
        TCHK(t, launch_round_weights(t->stream, t->net[f].w, t->net[f].q, t->net[f].w2b));
    std::vector<double> h(tail);
    TCHK(t, hipMemcpyAsync(h.data(), t->loss_hist, sizeof(double) * tail, hipMemcpyDeviceToHost, t->stream));
    TCHK(t, hipStreamSynchronize(t->stream));
    if (loss) {
        double s = 0.0;
        for (double v : h) s += v;
        *loss = s / (double)tail;
    }
    return MISA_OK;
}

}  // extern "C"
