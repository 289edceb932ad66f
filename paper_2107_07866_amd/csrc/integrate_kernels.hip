// Time integration (Sec. 2.1, Fig. 1: force, velocity and position update per
// step, read as kick-drift-kick velocity Verlet) fused with the first half of
// the hash update of Algorithm 2 (atoms farther than delta from their site
// leave the array), the adaptive step length, and the copies out of the store.
#include "misa_internal.h"

#include <algorithm>

namespace misa {

constexpr int KICK_BLOCKS = 1024;  // fixed grid => fixed reduction order
constexpr int KICK_THREADS = 256;

__device__ __forceinline__ double wave_sum_i(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max_i(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// v += (dt/2) C F / m;  u += dt v, from the current copy of u, v into the other
// (dst); an atom now farther than delta from its site is appended to this step's
// leavers and its slot emptied.  A leaver beyond the run-away capacity raises the
// overflow flag, and the run-away kick-drift that follows undoes the step.
template <typename Real>
__device__ __forceinline__ void kick_drift_body(State S, UV dst, Scratch sc, Geom g, double kf, int64_t rcap) {
    if (sc.cnt->overflow) return;  // frozen after an overflow: both copies hold the state
    const double dt = sc.scal[0];
    const double hk = 0.5 * dt * kf;
    const int64_t room = rcap - sc.cnt->n_run;
    const Real *fx = (const Real *)S.fx;
    const Real *fy = (const Real *)S.fy;
    const Real *fz = (const Real *)S.fz;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites;
         s += (int64_t)gridDim.x * blockDim.x) {
        // No branch before the arithmetic, so no load waits on another: an empty slot
        // (u = VACANT_U, v = 0, F = 0) comes out of the update unchanged and is only
        // kept out of the leaver test.
        double ux = S.ux[s], uy = S.uy[s], uz = S.uz[s];
        const bool vacant = ux > VACANT_TEST;
        const double vx = S.vx[s] + hk * (double)fx[s];
        const double vy = S.vy[s] + hk * (double)fy[s];
        const double vz = S.vz[s] + hk * (double)fz[s];
        ux += dt * vx;
        uy += dt * vy;
        uz += dt * vz;
        if (!vacant && ux * ux + uy * uy + uz * uz > g.delta2) {
            const int slot = atomicAdd(&sc.cnt->n_leave, 1);
            if (slot < room) {
                const int p = s >= g.ncell ? 1 : 0;
                const int64_t c = s - p * g.ncell;
                double sp[3];
                site_pos((int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny)), p, g.a, sp);
                sc.l_site[slot] = (int32_t)s;
                sc.l_id[slot] = S.atom[s];
                sc.l_x[slot] = wrap_coord(sp[0] + ux, g.L[0]);
                sc.l_y[slot] = wrap_coord(sp[1] + uy, g.L[1]);
                sc.l_z[slot] = wrap_coord(sp[2] + uz, g.L[2]);
                sc.l_vx[slot] = vx;
                sc.l_vy[slot] = vy;
                sc.l_vz[slot] = vz;
                dst.ux[s] = VACANT_U;
                dst.uy[s] = VACANT_U;
                dst.uz[s] = VACANT_U;
                dst.vx[s] = 0.0;
                dst.vy[s] = 0.0;
                dst.vz[s] = 0.0;
                S.atom[s] = VACANT_ID;
                continue;
            }
            atomicExch(&sc.cnt->overflow, 1);  // the step is undone before anything else reads it
        }
        dst.ux[s] = ux;
        dst.uy[s] = uy;
        dst.uz[s] = uz;
        dst.vx[s] = vx;
        dst.vy[s] = vy;
        dst.vz[s] = vz;
    }
}

template <typename Real>
__global__ __launch_bounds__(KICK_THREADS) void k_kick_drift(State S, UV dst, Scratch sc, Geom g, double kf,
                                                             int64_t rcap) {
    kick_drift_body<Real>(S, dst, sc, g, kf, rcap);
}

template <typename Real>
__global__ __launch_bounds__(KICK_THREADS) void kb_kick_drift(const BoxRef *__restrict__ boxes, double kf) {
    const BoxRef &B = boxes[blockIdx.y];
    kick_drift_body<Real>(B.S, B.alt, B.sc, B.g, kf, B.rcap);
}


// Run-away atoms: the same kick-drift, in place.  S is the copy the lattice
// kick-drift just wrote, prev the one it read.  After an overflow in that kick-drift
// this undoes the step instead: u, v of every site back from prev, the slots of the
// admitted leavers back to their atoms, and the run-away atoms stay where they were
// (the leaver count is cleared and dt set to zero by the leaver sort that follows).
__device__ __forceinline__ void kick_drift_runaway_body(State S, UV prev, Scratch sc, Geom g, double kf,
                                                        int64_t rcap) {
    const int ov = sc.cnt->overflow;
    if (ov == 1) {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites; s += stride) {
            S.ux[s] = prev.ux[s];
            S.uy[s] = prev.uy[s];
            S.uz[s] = prev.uz[s];
            S.vx[s] = prev.vx[s];
            S.vy[s] = prev.vy[s];
            S.vz[s] = prev.vz[s];
        }
        const int64_t room = rcap - sc.cnt->n_run;
        const int64_t nl = sc.cnt->n_leave < room ? sc.cnt->n_leave : room;
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nl; q += stride)
            S.atom[sc.l_site[q]] = sc.l_id[q];
        return;
    }
    if (ov) return;  // frozen
    const double dt = sc.scal[0];
    const double hk = 0.5 * dt * kf;
    const int n = sc.cnt->n_run;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const double vx = S.r_vx[r] + hk * S.r_fx[r];
        const double vy = S.r_vy[r] + hk * S.r_fy[r];
        const double vz = S.r_vz[r] + hk * S.r_fz[r];
        S.r_vx[r] = vx;
        S.r_vy[r] = vy;
        S.r_vz[r] = vz;
        S.r_x[r] = wrap_coord(S.r_x[r] + dt * vx, g.L[0]);
        S.r_y[r] = wrap_coord(S.r_y[r] + dt * vy, g.L[1]);
        S.r_z[r] = wrap_coord(S.r_z[r] + dt * vz, g.L[2]);
    }
}

__global__ void k_kick_drift_runaway(State S, UV prev, Scratch sc, Geom g, double kf, int64_t rcap) {
    kick_drift_runaway_body(S, prev, sc, g, kf, rcap);
}

// boxes: the box table after the swap (S the copy just written, alt the one read)
__global__ void kb_kick_drift_runaway(const BoxRef *__restrict__ boxes, double kf) {
    const BoxRef &B = boxes[blockIdx.y];
    kick_drift_runaway_body(B.S, B.alt, B.sc, B.g, kf, B.rcap);
}


// Second half-kick (kick = 1) or plain velocity statistics (kick = 0):
// per-block max |v|^2 and sum |v|^2 over the lattice atoms.
template <typename Real, bool kick>
__global__ __launch_bounds__(KICK_THREADS) void k_final_kick(State S, Scratch sc, Geom g, double kf,
                                                             double *__restrict__ part) {
    __shared__ double red[2][KICK_THREADS / 64];
    const double hk = 0.5 * sc.scal[0] * kf;
    const Real *fx = (const Real *)S.fx;
    const Real *fy = (const Real *)S.fy;
    const Real *fz = (const Real *)S.fz;
    double vm = 0.0, ks = 0.0;
    // An empty slot holds v = 0 and F = 0 (both cleared when it empties), so it
    // needs no test: its kick and its |v|^2 are zero.
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites;
         s += (int64_t)gridDim.x * blockDim.x) {
        double vx = S.vx[s], vy = S.vy[s], vz = S.vz[s];
        if (kick) {
            vx += hk * (double)fx[s];
            vy += hk * (double)fy[s];
            vz += hk * (double)fz[s];
            S.vx[s] = vx;
            S.vy[s] = vy;
            S.vz[s] = vz;
        }
        const double q = vx * vx + vy * vy + vz * vz;
        vm = fmax(vm, q);
        ks += q;
    }
    vm = wave_max_i(vm);
    ks = wave_sum_i(ks);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = vm;
        red[1][w] = ks;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < KICK_THREADS / 64; ++k) {
            a = fmax(a, red[0][k]);
            b += red[1][k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__device__ __forceinline__ void final_kick_runaway_body(State S, Scratch sc, double kf) {
    const double hk = 0.5 * sc.scal[0] * kf;
    const int n = sc.cnt->n_run;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        S.r_vx[r] += hk * S.r_fx[r];
        S.r_vy[r] += hk * S.r_fy[r];
        S.r_vz[r] += hk * S.r_fz[r];
    }
}

__global__ void k_final_kick_runaway(State S, Scratch sc, double kf) {
    final_kick_runaway_body(S, sc, kf);
}

__global__ void kb_final_kick_runaway(const BoxRef *__restrict__ boxes, double kf) {
    const BoxRef &B = boxes[blockIdx.y];
    final_kick_runaway_body(B.S, B.sc, kf);
}


// max |v|, kinetic energy, and the next step length
// dt = min(dt_max, dx_max / max|v|)  (dx_max <= 0: dt = dt_max).
// use_aff: lattice atoms next to run-aways were left out of the per-tile partials of
// the fused kick; their |v|^2 come from the (sorted) affected list.
__device__ __forceinline__ void dt_update_body(State S, Scratch sc, const double *__restrict__ part, int nblk,
                                                    int use_aff, double mass, double dt_max, double dx_max,
                                                    int first) {
    __shared__ double red[2][1024 / 64];
    if (!first && sc.cnt->overflow) return;  // frozen after an overflow: dt stays zero, time stands still
    double vm = 0.0, ks = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 1024) {
        vm = fmax(vm, part[2 * i]);
        ks += part[2 * i + 1];
    }
    if (use_aff) {
        int na = sc.cnt->n_affected;
        na = na < sc.affected_cap ? na : (int)sc.affected_cap;
        for (int q = threadIdx.x; q < na; q += 1024) {
            vm = fmax(vm, sc.aff_v2[q]);
            ks += sc.aff_v2[q];
        }
    }
    const int n = sc.cnt->n_run;
    for (int r = threadIdx.x; r < n; r += 1024) {
        const double q = S.r_vx[r] * S.r_vx[r] + S.r_vy[r] * S.r_vy[r] + S.r_vz[r] * S.r_vz[r];
        vm = fmax(vm, q);
        ks += q;
    }
    vm = wave_max_i(vm);
    ks = wave_sum_i(ks);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = vm;
        red[1][w] = ks;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 1024 / 64; ++k) {
            a = fmax(a, red[0][k]);
            b += red[1][k];
        }
        const double vmax = sqrt(a);
        double dt = dt_max;
        if (dx_max > 0.0 && vmax > 0.0 && dx_max / vmax < dt_max) dt = dx_max / vmax;
        if (!first) {
            sc.scal[1] += sc.scal[0];
            sc.scal[6] = sc.scal[0];
            sc.cnt->steps += 1;
        } else {  // a new call: no overflow, no steps yet
            sc.cnt->overflow = 0;
            sc.cnt->steps = 0;
            sc.cnt->fail_step = 0;
        }
        sc.scal[0] = dt;
        sc.scal[2] = vmax;
        sc.scal[3] = 0.5 * mass * b / ACC_UNIT;
    }
}

__global__ __launch_bounds__(1024) void k_dt_update(State S, Scratch sc, const double *__restrict__ part, int nblk,
                                                    int use_aff, double mass, double dt_max, double dx_max,
                                                    int first) {
    dt_update_body(S, sc, part, nblk, use_aff, mass, dt_max, dx_max, first);
}

__global__ __launch_bounds__(1024) void kb_dt_update(const BoxRef *__restrict__ boxes, double mass, double dt_max, double dx_max) {
    const BoxRef &B = boxes[blockIdx.y];
    dt_update_body(B.S, B.sc, B.sc.part_kick, B.g.ntiles2, 1, mass, dt_max, dx_max, 0);
}


// ---------------------------------------------------------------------------
// placement into the store (misa_set_state): the hash rule of Sec. 3 applied to
// every atom at once.  An atom takes the slot of its nearest site when it lies
// within delta of it and no lower atom id claims the same slot; every other atom
// becomes a run-away atom (listed afterwards in ascending id by the leaver sort
// and compaction of the hash update).

template <typename Real>
__global__ void k_place_clear(State S, Geom g) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites; s += stride) {
        S.atom[s] = VACANT_ID;
        S.ux[s] = VACANT_U;
        S.uy[s] = VACANT_U;
        S.uz[s] = VACANT_U;
        S.vx[s] = 0.0;
        S.vy[s] = 0.0;
        S.vz[s] = 0.0;
        ((Real *)S.fx)[s] = (Real)0;
        ((Real *)S.fy)[s] = (Real)0;
        ((Real *)S.fz)[s] = (Real)0;
        ((Real *)S.rho)[s] = (Real)0;
        ((Real *)S.fp)[s] = (Real)0;
    }
}

// Bids: atom i within delta of its nearest site bids for that slot with its id.
// x, v: (n, 3) row-major device arrays; bad counts non-finite inputs.
__global__ void k_place_claim(const double *__restrict__ x, const double *__restrict__ v, int64_t n, Geom g,
                              State S, int32_t *__restrict__ cand, uint32_t *__restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double X[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        const double V[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        bool finite = true;
        for (int k = 0; k < 3; ++k) finite = finite && isfinite(X[k]) && isfinite(V[k]);
        int32_t c = -1;
        if (!finite) {
            atomicAdd(bad, 1u);
        } else {
            double u[3], u2;
            const int64_t s = hash_site(X, g, u, &u2);
            if (u2 <= g.delta2) {
                c = (int32_t)s;
                atomicMin(&S.atom[s], (int32_t)i);
            }
        }
        cand[i] = c;
    }
}

// The lowest bidder moves into its slot; every other atom joins the leaver list
// (capacity rcap; the count keeps growing past it so the host can report it).
__global__ void k_place_settle(const double *__restrict__ x, const double *__restrict__ v, int64_t n, Geom g,
                               State S, Scratch sc, const int32_t *__restrict__ cand, int64_t rcap) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double X[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        const double V[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        const int32_t s = cand[i];
        if (s >= 0 && S.atom[s] == (int32_t)i) {
            double u[3], u2;
            hash_site(X, g, u, &u2);
            S.ux[s] = u[0];
            S.uy[s] = u[1];
            S.uz[s] = u[2];
            S.vx[s] = V[0];
            S.vy[s] = V[1];
            S.vz[s] = V[2];
        } else {
            const int slot = atomicAdd(&sc.cnt->n_leave, 1);
            if (slot < rcap) {
                sc.l_site[slot] = -1;
                sc.l_id[slot] = (int32_t)i;
                sc.l_x[slot] = wrap_coord(X[0], g.L[0]);
                sc.l_y[slot] = wrap_coord(X[1], g.L[1]);
                sc.l_z[slot] = wrap_coord(X[2], g.L[2]);
                sc.l_vx[slot] = V[0];
                sc.l_vy[slot] = V[1];
                sc.l_vz[slot] = V[2];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// copies out of the store, in atom-id order

__global__ void k_gather_state(State S, Scratch sc, Geom g, double *__restrict__ x, double *__restrict__ v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites; s += stride) {
        const int32_t id = S.atom[s];
        if (id == VACANT_ID) continue;
        if (x) {
            const int p = s >= g.ncell ? 1 : 0;
            const int64_t c = s - p * g.ncell;
            double sp[3];
            site_pos((int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny)), p, g.a, sp);
            x[3 * (int64_t)id] = wrap_coord(sp[0] + S.ux[s], g.L[0]);
            x[3 * (int64_t)id + 1] = wrap_coord(sp[1] + S.uy[s], g.L[1]);
            x[3 * (int64_t)id + 2] = wrap_coord(sp[2] + S.uz[s], g.L[2]);
        }
        if (v) {
            v[3 * (int64_t)id] = S.vx[s];
            v[3 * (int64_t)id + 1] = S.vy[s];
            v[3 * (int64_t)id + 2] = S.vz[s];
        }
    }
    const int n = sc.cnt->n_run;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const int64_t id = S.r_id[r];
        if (x) {
            x[3 * id] = S.r_x[r];
            x[3 * id + 1] = S.r_y[r];
            x[3 * id + 2] = S.r_z[r];
        }
        if (v) {
            v[3 * id] = S.r_vx[r];
            v[3 * id + 1] = S.r_vy[r];
            v[3 * id + 2] = S.r_vz[r];
        }
    }
}

template <typename Real>
__global__ void k_gather_field(State S, Scratch sc, Geom g, int field, double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const Real *rho = (const Real *)S.rho;
    const Real *fp = (const Real *)S.fp;
    const Real *fx = (const Real *)S.fx;
    const Real *fy = (const Real *)S.fy;
    const Real *fz = (const Real *)S.fz;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites; s += stride) {
        const int32_t id = S.atom[s];
        if (id == VACANT_ID) continue;
        if (field == MISA_FIELD_RHO) out[id] = (double)rho[s];
        else if (field == MISA_FIELD_FPRIME) out[id] = (double)fp[s];
        else {
            out[3 * (int64_t)id] = (double)fx[s];
            out[3 * (int64_t)id + 1] = (double)fy[s];
            out[3 * (int64_t)id + 2] = (double)fz[s];
        }
    }
    const int n = sc.cnt->n_run;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const int64_t id = S.r_id[r];
        if (field == MISA_FIELD_RHO) out[id] = S.r_rho[r];
        else if (field == MISA_FIELD_FPRIME) out[id] = S.r_fp[r];
        else {
            out[3 * id] = S.r_fx[r];
            out[3 * id + 1] = S.r_fy[r];
            out[3 * id + 2] = S.r_fz[r];
        }
    }
}

__global__ void k_gather_slots(State S, Scratch sc, Geom g, int64_t *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites; s += stride) {
        const int32_t id = S.atom[s];
        if (id != VACANT_ID) out[id] = lattice_id_of(s, g);
    }
    const int n = sc.cnt->n_run;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) out[S.r_id[r]] = -1;
}

// ---------------------------------------------------------------------------
// launchers

static int site_blocks(const Geom &g) {
    int64_t b = (g.nsites + KICK_THREADS - 1) / KICK_THREADS;
    return (int)(b < 65536 * 4 ? (b > 0 ? b : 1) : 65536 * 4);
}

void swap_uv(misa_lattice *h) {
    std::swap(h->S.ux, h->alt.ux);
    std::swap(h->S.uy, h->alt.uy);
    std::swap(h->S.uz, h->alt.uz);
    std::swap(h->S.vx, h->alt.vx);
    std::swap(h->S.vy, h->alt.vy);
    std::swap(h->S.vz, h->alt.vz);
    h->parity ^= 1;
}

hipError_t launch_kick_drift(misa_lattice *h) {
    const double kf = ACC_UNIT / h->mass;
    const int nb = site_blocks(h->g);
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_kick_drift<float>, dim3(nb), dim3(KICK_THREADS), 0, h->stream, h->S, h->alt, h->sc, h->g,
                           kf, h->rcap);
    else
        hipLaunchKernelGGL(k_kick_drift<double>, dim3(nb), dim3(KICK_THREADS), 0, h->stream, h->S, h->alt, h->sc,
                           h->g, kf, h->rcap);
    swap_uv(h);
    hipLaunchKernelGGL(k_kick_drift_runaway, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->S, h->alt, h->sc, h->g, kf,
                       h->rcap);
    return hipGetLastError();
}

static hipError_t kick_impl(misa_lattice *h, int kick) {
    const double kf = ACC_UNIT / h->mass;
    double *part = h->sc.part + 2 * (int64_t)h->g.ntiles_pad;  // after the per-tile energy partials
    auto kern = h->precision == MISA_FP32 ? (kick ? k_final_kick<float, true> : k_final_kick<float, false>)
                                          : (kick ? k_final_kick<double, true> : k_final_kick<double, false>);
    hipLaunchKernelGGL(kern, dim3(KICK_BLOCKS), dim3(KICK_THREADS), 0, h->stream, h->S, h->sc, h->g, kf, part);
    if (kick)
        hipLaunchKernelGGL(k_final_kick_runaway, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->S, h->sc, kf);
    return hipGetLastError();
}

hipError_t launch_final_kick(misa_lattice *h) {
    if (!fused_kick(h)) return kick_impl(h, 1);
    // lattice atoms were kicked inside the force pass; only run-away atoms remain
    hipLaunchKernelGGL(k_final_kick_runaway, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->S, h->sc,
                       ACC_UNIT / h->mass);
    return hipGetLastError();
}

hipError_t launch_dt_update(misa_lattice *h, double dt_max, double dx_max, bool first) {
    if (first) {
        hipError_t e = kick_impl(h, 0);
        if (e != hipSuccess) return e;
    }
    const bool fused = fused_kick(h) && !first;
    const double *part = fused ? h->sc.part_kick : h->sc.part + 2 * (int64_t)h->g.ntiles_pad;
    // per-tile partials of the force pass that kicked: persistent tiles or generic tiles
    const int nblk = fused ? (force_on_tiles2(h) ? h->g.ntiles2 : h->g.ntiles) : KICK_BLOCKS;
    hipLaunchKernelGGL(k_dt_update, dim3(1), dim3(1024), 0, h->stream, h->S, h->sc, part, nblk, fused ? 1 : 0,
                       h->mass, dt_max, dx_max, first ? 1 : 0);
    return hipGetLastError();
}

// Batched: one launch per kernel over every box (blockIdx.y = box).
hipError_t launchb_kick_drift(hipStream_t st, const BoxRef *boxes, const BoxRef *boxes_after, int nbox, int gx_sites,
                              int gx_small, double kf) {
    hipLaunchKernelGGL(kb_kick_drift<float>, dim3(gx_sites, nbox), dim3(KICK_THREADS), 0, st, boxes, kf);
    hipLaunchKernelGGL(kb_kick_drift_runaway, dim3(gx_small, nbox), dim3(256), 0, st, boxes_after, kf);
    return hipGetLastError();
}

hipError_t launchb_final_kick_runaway(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small, double kf) {
    hipLaunchKernelGGL(kb_final_kick_runaway, dim3(gx_small, nbox), dim3(256), 0, st, boxes, kf);
    return hipGetLastError();
}

hipError_t launchb_dt_update(hipStream_t st, const BoxRef *boxes, int nbox, double mass, double dt_max,
                             double dx_max) {
    hipLaunchKernelGGL(kb_dt_update, dim3(1, nbox), dim3(1024), 0, st, boxes, mass, dt_max, dx_max);
    return hipGetLastError();
}

hipError_t launch_place(misa_lattice *h, const double *x, const double *v, int64_t n, int32_t *cand,
                        uint32_t *bad) {
    const int nb = site_blocks(h->g);
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_place_clear<float>, dim3(nb), dim3(KICK_THREADS), 0, h->stream, h->S, h->g);
    else
        hipLaunchKernelGGL(k_place_clear<double>, dim3(nb), dim3(KICK_THREADS), 0, h->stream, h->S, h->g);
    if (n > 0) {
        const int na = (int)std::min<int64_t>((n + KICK_THREADS - 1) / KICK_THREADS, 65536 * 4);
        hipLaunchKernelGGL(k_place_claim, dim3(na), dim3(KICK_THREADS), 0, h->stream, x, v, n, h->g, h->S, cand,
                           bad);
        hipLaunchKernelGGL(k_place_settle, dim3(na), dim3(KICK_THREADS), 0, h->stream, x, v, n, h->g, h->S, h->sc,
                           cand, h->rcap);
    }
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, uint32_t value, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = value;
}

hipError_t launch_fill_u32(misa_lattice *h, uint32_t *a, uint32_t value, int64_t n) {
    const int nb = (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, h->stream, a, value, n);
    return hipGetLastError();
}

hipError_t launch_gather_state(misa_lattice *h, double *x, double *v) {
    hipLaunchKernelGGL(k_gather_state, dim3(site_blocks(h->g)), dim3(KICK_THREADS), 0, h->stream, h->S, h->sc, h->g,
                       x, v);
    return hipGetLastError();
}

hipError_t launch_gather_field(misa_lattice *h, int field, double *out) {
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_gather_field<float>, dim3(site_blocks(h->g)), dim3(KICK_THREADS), 0, h->stream, h->S,
                           h->sc, h->g, field, out);
    else
        hipLaunchKernelGGL(k_gather_field<double>, dim3(site_blocks(h->g)), dim3(KICK_THREADS), 0, h->stream, h->S,
                           h->sc, h->g, field, out);
    return hipGetLastError();
}

hipError_t launch_gather_slots(misa_lattice *h, int64_t *out) {
    hipLaunchKernelGGL(k_gather_slots, dim3(site_blocks(h->g)), dim3(KICK_THREADS), 0, h->stream, h->S, h->sc, h->g,
                       out);
    return hipGetLastError();
}

}  // namespace misa
