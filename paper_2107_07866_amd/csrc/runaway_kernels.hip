// Atoms outside the lattice array (the hash-clash atoms of Sec. 3):
//   - hash update (Algorithm 2): atoms that drifted more than delta from their
//     site leave the array; run-away atoms take the empty slot of their nearest
//     site when within delta of it (lowest atom id wins, via atomicMin on the
//     slot's id word);
//   - a device hash of run-away atoms bucketed by coarse cells (edge >= rc):
//     atoms sorted by (cell, list index), open-addressing map cell -> first
//     position;
//   - run-away interactions (Algorithm 1, second and third loops) with every
//     unordered pair counted on both ends: a run-away atom gathers from lattice
//     sites in a window around it and from other run-aways through the hash;
//     each lattice atom within rc of a run-away gathers the matching reaction
//     terms itself, with the pair vector computed bit-identically, so no
//     scatter, atomics on floats or colouring are needed and results are
//     deterministic run to run.
// All arithmetic here is float64 regardless of the lattice pair precision.
#include "misa_internal.h"

namespace misa {

// ---------------------------------------------------------------------------
// helpers

__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename Real>
__device__ __forceinline__ void seg64(double x, const TabMeta<Real> &m, int &k, double &t) {
    const double p = (x - (double)m.x0) * (double)m.inv_h;
    int kk = (int)p;
    kk = kk < m.nseg - 1 ? kk : m.nseg - 1;
    kk = kk > 0 ? kk : 0;
    k = kk;
    t = p - (double)kk;
}

__device__ __forceinline__ double f_val(double r, const Tables<double> &T) {
    int k;
    double t;
    seg64(r, T.fm, k, t);
    const Q4<double> c = T.f[k];
    return ((c.w * t + c.z) * t + c.y) * t + c.x;
}

// f'(r), phi'(r) and phi(r)
__device__ __forceinline__ void fp_phi(double r, const Tables<double> &T, double &df, double &dphi, double &phi) {
    int k;
    double t;
    seg64(r, T.fm, k, t);
    const Q4<double> a = T.force[2 * k];
    const Q4<double> b = T.force[2 * k + 1];
    const Q4<double> c = T.phi[k];
    df = (a.z * t + a.y) * t + a.x;
    dphi = (b.y * t + b.x) * t + a.w;
    phi = ((c.w * t + c.z) * t + c.y) * t + c.x;
}

template <typename Real>
__device__ __forceinline__ Real emb_any(Real rho, const Q4<Real> *__restrict__ emb, const TabMeta<Real> &m,
                                        Real &Fval, bool &beyond) {
    if (rho > m.x_last) {
        beyond = true;
        Fval = m.y_last + m.d_last * (rho - m.x_last);
        return m.d_last;
    }
    const Real p = (rho - m.x0) * m.inv_h;
    int k = (int)p;
    k = k < m.nseg - 1 ? k : m.nseg - 1;
    k = k > 0 ? k : 0;
    Real t = p - (Real)k;
    const Q4<Real> c = emb[2 * k];
    const Q4<Real> d = emb[2 * k + 1];
    Fval = ((c.w * t + c.z) * t + c.y) * t + c.x;
    return (d.z * t + d.y) * t + d.x;
}

__device__ __forceinline__ uint32_t hash_slot(int32_t key, int32_t mask) {
    uint32_t h = (uint32_t)key * 2654435761u;
    return (h ^ (h >> 16)) & (uint32_t)mask;
}

__device__ __forceinline__ int32_t hash_find(int32_t key, const int32_t *__restrict__ hkey,
                                             const int32_t *__restrict__ hval, int32_t mask) {
    uint32_t h = hash_slot(key, mask);
    for (int probe = 0; probe <= mask; ++probe) {
        const int32_t k = hkey[h];
        if (k == key) return hval[h];
        if (k == -1) return -1;
        h = (h + 1) & (uint32_t)mask;
    }
    return -1;
}

__device__ __forceinline__ int coarse_of(double xw, int nc, double inv_cs) {
    int c = (int)(xw * inv_cs);
    return c >= nc ? nc - 1 : (c < 0 ? 0 : c);
}

__device__ __forceinline__ int axis_cells(int c, int n, int out[3]) {
    if (n == 1) {
        out[0] = 0;
        return 1;
    }
    if (n == 2) {
        out[0] = 0;
        out[1] = 1;
        return 2;
    }
    out[0] = c == 0 ? n - 1 : c - 1;
    out[1] = c;
    out[2] = c == n - 1 ? 0 : c + 1;
    return 3;
}

// First cell of the lattice window searched around a run-away atom at q = x / a:
// every integer c with c > q - reach - 1/2 (covers corner sites c and centre sites c + 1/2).
__device__ __forceinline__ int window_lo(double q, double reach) { return (int)floor(q - reach - 0.5) + 1; }

// Separation x_j - x_r of lattice atom (site cell cx,cy,cz unwrapped near the
// run-away, sublattice p, displacement u) from run-away atom x: computed the same
// way by both kernels that see this pair.
__device__ __forceinline__ void lat_sep(int cx, int cy, int cz, int p, const double u[3], const double x[3],
                                        double a, double d[3]) {
    double sp[3];
    site_pos(cx, cy, cz, p, a, sp);
    d[0] = (sp[0] - x[0]) + u[0];
    d[1] = (sp[1] - x[1]) + u[1];
    d[2] = (sp[2] - x[2]) + u[2];
}

__device__ __forceinline__ void min_image3(double d[3], const Geom &g) {
    for (int k = 0; k < 3; ++k) d[k] -= g.L[k] * rint(d[k] / g.L[k]);
}

// ---------------------------------------------------------------------------
// single-block bitonic sort of 64-bit keys (ascending); mode 0: leavers by atom
// id, mode 1: run-aways by (coarse cell, list index)

__global__ __launch_bounds__(SORT_THREADS) void k_sort(uint64_t *__restrict__ buf, int mode,
                                                        Counters *__restrict__ cnt, int64_t rcap,
                                                        const int32_t *__restrict__ l_id,
                                                        const double *__restrict__ rx, const double *__restrict__ ry,
                                                        const double *__restrict__ rz, Geom g) {
    __shared__ uint64_t sh[SORT_LDS_MAX];
    int n;
    if (mode == 0) {
        // leavers beyond the run-away capacity were not recorded (they kept their slots)
        const int nl = cnt->n_leave;
        const int room = (int)(rcap - cnt->n_run);
        n = nl < room ? nl : room;
    } else {
        n = cnt->n_run;
    }
    __syncthreads();
    if (mode == 0 && threadIdx.x == 0) cnt->n_leave = n;
    if (n <= 1) {
        if (n == 1 && threadIdx.x == 0) {
            if (mode == 0) {
                buf[0] = ((uint64_t)(uint32_t)l_id[0] << 32) | 0u;
            } else {
                int kx = coarse_of(rx[0], g.nc[0], g.inv_cs[0]);
                int ky = coarse_of(ry[0], g.nc[1], g.inv_cs[1]);
                int kz = coarse_of(rz[0], g.nc[2], g.inv_cs[2]);
                int32_t key = (kz * g.nc[1] + ky) * g.nc[0] + kx;
                buf[0] = ((uint64_t)(uint32_t)key << 32) | 0u;
            }
        }
        return;
    }
    int P = 1;
    while (P < n) P <<= 1;
    const bool in_lds = P <= SORT_LDS_MAX;
    uint64_t *A = in_lds ? sh : buf;
    for (int i = threadIdx.x; i < P; i += SORT_THREADS) {
        uint64_t v = ~0ull;
        if (i < n) {
            if (mode == 0) {
                v = ((uint64_t)(uint32_t)l_id[i] << 32) | (uint32_t)i;
            } else {
                int kx = coarse_of(rx[i], g.nc[0], g.inv_cs[0]);
                int ky = coarse_of(ry[i], g.nc[1], g.inv_cs[1]);
                int kz = coarse_of(rz[i], g.nc[2], g.inv_cs[2]);
                int32_t key = (kz * g.nc[1] + ky) * g.nc[0] + kx;
                v = ((uint64_t)(uint32_t)key << 32) | (uint32_t)i;
            }
        }
        A[i] = v;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += SORT_THREADS) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = A[i], b = A[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        A[i] = b;
                        A[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (in_lds)
        for (int i = threadIdx.x; i < n; i += SORT_THREADS) buf[i] = sh[i];
}

// ---------------------------------------------------------------------------
// hash update

// Claims: each run-away atom and each leaver of this step that lies within
// delta of its nearest site, and finds that slot empty, bids with its atom id.
__global__ void k_claim(State S, Scratch sc, Geom g) {
    const int nrun = sc.cnt->n_run;
    const int total = nrun + sc.cnt->n_leave;  // leavers admitted this step (clamped by k_sort)
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        double x[3];
        int32_t id;
        if (q < nrun) {
            x[0] = S.r_x[q];
            x[1] = S.r_y[q];
            x[2] = S.r_z[q];
            id = S.r_id[q];
        } else {
            const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
            x[0] = sc.l_x[li];
            x[1] = sc.l_y[li];
            x[2] = sc.l_z[li];
            id = sc.l_id[li];
        }
        double u[3], u2;
        const int64_t s = hash_site(x, g, u, &u2);
        int32_t cand = -1;
        if (u2 <= g.delta2 && S.ux[s] > VACANT_TEST) {
            cand = (int32_t)s;
            atomicMin(&S.atom[s], id);
        }
        sc.cand[q] = cand;
    }
}

// The lowest bidder of each contested slot moves in.
__global__ void k_settle(State S, Scratch sc, Geom g) {
    const int nrun = sc.cnt->n_run;
    const int total = nrun + sc.cnt->n_leave;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int32_t s = sc.cand[q];
        uint8_t done = 0;
        if (s >= 0) {
            double x[3], v[3];
            int32_t id;
            if (q < nrun) {
                x[0] = S.r_x[q];
                x[1] = S.r_y[q];
                x[2] = S.r_z[q];
                v[0] = S.r_vx[q];
                v[1] = S.r_vy[q];
                v[2] = S.r_vz[q];
                id = S.r_id[q];
            } else {
                const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
                x[0] = sc.l_x[li];
                x[1] = sc.l_y[li];
                x[2] = sc.l_z[li];
                v[0] = sc.l_vx[li];
                v[1] = sc.l_vy[li];
                v[2] = sc.l_vz[li];
                id = sc.l_id[li];
            }
            if (S.atom[s] == id) {
                double u[3], u2;
                hash_site(x, g, u, &u2);
                S.ux[s] = u[0];
                S.uy[s] = u[1];
                S.uz[s] = u[2];
                S.vx[s] = v[0];
                S.vy[s] = v[1];
                S.vz[s] = v[2];
                done = 1;
            }
        }
        sc.settled[q] = done;
    }
}

// Stable compaction: surviving run-aways keep their order, surviving leavers
// follow in ascending atom id.  Single work-group.
__global__ __launch_bounds__(1024) void k_compact(State S, Scratch sc) {
    __shared__ int wsum[1024 / 64];
    __shared__ int base_sh;
    const int nrun = sc.cnt->n_run;
    const int nl = sc.cnt->n_leave;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    const int total = nrun + nl;
    for (int c0 = 0; c0 < total; c0 += 1024) {
        const int q = c0 + threadIdx.x;
        const bool keep = q < total && !sc.settled[q];
        int32_t id = 0;
        double x = 0, y = 0, z = 0, vx = 0, vy = 0, vz = 0;
        if (keep) {
            if (q < nrun) {
                id = S.r_id[q];
                x = S.r_x[q];
                y = S.r_y[q];
                z = S.r_z[q];
                vx = S.r_vx[q];
                vy = S.r_vy[q];
                vz = S.r_vz[q];
            } else {
                const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
                id = sc.l_id[li];
                x = sc.l_x[li];
                y = sc.l_y[li];
                z = sc.l_z[li];
                vx = sc.l_vx[li];
                vy = sc.l_vy[li];
                vz = sc.l_vz[li];
            }
        }
        const uint64_t m = __ballot(keep);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(m);
        __syncthreads();
        int off = base_sh;
        for (int k = 0; k < w; ++k) off += wsum[k];
        int tot = 0;
        for (int k = 0; k < 1024 / 64; ++k) tot += wsum[k];
        __syncthreads();  // every lane has read its record and the wave sums
        if (keep) {
            const int o = off + below;
            S.r_id[o] = id;
            S.r_x[o] = x;
            S.r_y[o] = y;
            S.r_z[o] = z;
            S.r_vx[o] = vx;
            S.r_vy[o] = vy;
            S.r_vz[o] = vz;
        }
        if (threadIdx.x == 0) base_sh += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc.cnt->n_run = base_sh;
        sc.cnt->n_leave = 0;
    }
}

// ---------------------------------------------------------------------------
// device hash of run-away atoms

__global__ void k_hash_insert(Scratch sc) {
    const int n = sc.cnt->n_run;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const uint64_t v = sc.sortbuf[q];
        const int32_t key = (int32_t)(v >> 32);
        sc.skey[q] = key;
        sc.sidx[q] = (int32_t)(v & 0xffffffffu);
        const bool start = q == 0 || (int32_t)(sc.sortbuf[q - 1] >> 32) != key;
        if (start) {
            uint32_t h = hash_slot(key, sc.hmask);
            for (int probe = 0; probe <= sc.hmask; ++probe) {
                if (atomicCAS(&sc.hkey[h], -1, key) == -1) {
                    sc.hval[h] = q;
                    sc.hslot[q] = (int32_t)h;
                    break;
                }
                h = (h + 1) & (uint32_t)sc.hmask;
            }
        }
    }
}

__global__ void k_hash_clear(Scratch sc) {
    const int n = sc.cnt->n_run;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const bool start = q == 0 || sc.skey[q - 1] != sc.skey[q];
        if (start) sc.hkey[sc.hslot[q]] = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sc.cnt->n_affected = 0;
}

// Run-away atoms (list positions, ascending) closer than sqrt(cut2) to position x,
// found through the hash.  Calls fn(o, d, r2) with d = x_o - x (minimum image).
template <typename Fn>
__device__ __forceinline__ void for_runaway_neighbours(const double x[3], int self, int lane, int step,
                                                       double cut2, const State &S, const Scratch &sc,
                                                       const Geom &g, Fn fn) {
    const int n = sc.cnt->n_run;
    int cx[3], cy[3], cz[3];
    const int nxc = axis_cells(coarse_of(x[0], g.nc[0], g.inv_cs[0]), g.nc[0], cx);
    const int nyc = axis_cells(coarse_of(x[1], g.nc[1], g.inv_cs[1]), g.nc[1], cy);
    const int nzc = axis_cells(coarse_of(x[2], g.nc[2], g.inv_cs[2]), g.nc[2], cz);
    for (int az = 0; az < nzc; ++az)
        for (int ay = 0; ay < nyc; ++ay)
            for (int ax = 0; ax < nxc; ++ax) {
                const int32_t key = (cz[az] * g.nc[1] + cy[ay]) * g.nc[0] + cx[ax];
                const int32_t start = hash_find(key, sc.hkey, sc.hval, sc.hmask);
                if (start < 0) continue;
                for (int q = start + lane; q < n && sc.skey[q] == key; q += step) {
                    const int o = sc.sidx[q];
                    if (o == self) continue;
                    double d[3] = {S.r_x[o] - x[0], S.r_y[o] - x[1], S.r_z[o] - x[2]};
                    min_image3(d, g);
                    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (r2 < cut2) fn(o, d, r2);
                }
            }
}

// ---------------------------------------------------------------------------
// densities

// One wave per run-away atom: rho from lattice sites in its window and from other
// run-aways; marks every lattice atom it pairs with (they need the reaction term).
__global__ __launch_bounds__(64 * RUNAWAY_WAVES_PER_BLOCK) void k_runaway_rho(State S, Scratch sc, Geom g,
                                                                              Tables<double> T) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * RUNAWAY_WAVES_PER_BLOCK + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * RUNAWAY_WAVES_PER_BLOCK;
    const int n = sc.cnt->n_run;
    const int win = g.win, win3 = win * win * win;
    for (int r = wave; r < n; r += nwaves) {
        const double x[3] = {S.r_x[r], S.r_y[r], S.r_z[r]};
        const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                           window_lo(x[2] * g.inv_a, g.reach)};
        double acc = 0.0;
        for (int c = lane; c < 2 * win3; c += 64) {
            const int p = c >= win3 ? 1 : 0;
            const int rem = c - p * win3;
            const int cx = lo[0] + rem % win, cy = lo[1] + (rem / win) % win, cz = lo[2] + rem / (win * win);
            const int64_t s = (int64_t)p * g.ncell +
                              ((int64_t)wrap_index(cz, g.nz) * g.ny + wrap_index(cy, g.ny)) * g.nx +
                              wrap_index(cx, g.nx);
            const double ux = S.ux[s];
            if (ux > VACANT_TEST) continue;
            const double u[3] = {ux, S.uy[s], S.uz[s]};
            double d[3];
            lat_sep(cx, cy, cz, p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) {
                acc += f_val(sqrt(r2), T);
                const uint32_t bit = 1u << (s & 31);
                const uint32_t old = atomicOr(&sc.mark[s >> 5], bit);
                if (!(old & bit)) {
                    const int pos = atomicAdd(&sc.cnt->n_affected, 1);
                    if (pos < sc.affected_cap)
                        sc.affected[pos] = (int32_t)s;
                    else
                        atomicExch(&sc.cnt->overflow, 1);
                }
            }
        }
        for_runaway_neighbours(x, r, lane, 64, g.rc2, S, sc, g,
                               [&](int, const double *, double r2) { acc += f_val(sqrt(r2), T); });
        acc = wave_sum64(acc);
        if (lane == 0) {
            double Fv;
            bool beyond = false;
            const double d = emb_any<double>(acc, T.emb, T.em, Fv, beyond);
            S.r_rho[r] = acc;
            S.r_fp[r] = d;
            S.r_e[2 * r] = Fv;
            if (beyond) atomicAdd(&sc.cnt->range_viol, 1u);
        }
    }
}

// Lattice atoms within rc of run-aways: add the run-away terms to rho, refresh F'.
template <typename Real>
__global__ void k_affected_rho(State S, Scratch sc, Geom g, Tables<double> T, Tables<Real> TL) {
    int na = sc.cnt->n_affected;
    na = na < sc.affected_cap ? na : (int)sc.affected_cap;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < na; q += gridDim.x * blockDim.x) {
        const int64_t s = sc.affected[q];
        const int p = s >= g.ncell ? 1 : 0;
        const int64_t c = s - p * g.ncell;
        const int cxj = (int)(c % g.nx), cyj = (int)((c / g.nx) % g.ny), czj = (int)(c / ((int64_t)g.nx * g.ny));
        const double u[3] = {S.ux[s], S.uy[s], S.uz[s]};
        double xj[3];
        site_pos(cxj, cyj, czj, p, g.a, xj);
        for (int k = 0; k < 3; ++k) xj[k] = wrap_coord(xj[k] + u[k], g.L[k]);
        double acc = 0.0;
        // candidates through the hash (generous test), exact pair test as the run-away saw it
        for_runaway_neighbours(xj, -1, 0, 1, g.pre2, S, sc, g, [&](int o, const double *, double) {
            const double x[3] = {S.r_x[o], S.r_y[o], S.r_z[o]};
            int cc[3];
            const int cj[3] = {cxj, cyj, czj};
            const int nn[3] = {g.nx, g.ny, g.nz};
            for (int k = 0; k < 3; ++k) {
                const int lo = window_lo(x[k] * g.inv_a, g.reach);
                cc[k] = lo + wrap_index(cj[k] - lo, nn[k]);
                if (cc[k] - lo >= g.win) return;
            }
            double d[3];
            lat_sep(cc[0], cc[1], cc[2], p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) acc += f_val(sqrt(r2), T);
        });
        Real *rho = (Real *)S.rho;
        Real *fp = (Real *)S.fp;
        const Real rj = rho[s] + (Real)acc;
        rho[s] = rj;
        Real Fv;
        bool beyond = false;
        fp[s] = emb_any<Real>(rj, TL.emb, TL.em, Fv, beyond);
        if (beyond) atomicAdd(&sc.cnt->range_viol, 1u);
    }
}

// ---------------------------------------------------------------------------
// forces

__global__ __launch_bounds__(64 * RUNAWAY_WAVES_PER_BLOCK) void k_runaway_force(State S, Scratch sc, Geom g,
                                                                                Tables<double> T, int real_is_f32,
                                                                                int energy) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * RUNAWAY_WAVES_PER_BLOCK + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * RUNAWAY_WAVES_PER_BLOCK;
    const int n = sc.cnt->n_run;
    const int win = g.win, win3 = win * win * win;
    for (int r = wave; r < n; r += nwaves) {
        const double x[3] = {S.r_x[r], S.r_y[r], S.r_z[r]};
        const double fpr = S.r_fp[r];
        const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                           window_lo(x[2] * g.inv_a, g.reach)};
        double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
        for (int c = lane; c < 2 * win3; c += 64) {
            const int p = c >= win3 ? 1 : 0;
            const int rem = c - p * win3;
            const int cx = lo[0] + rem % win, cy = lo[1] + (rem / win) % win, cz = lo[2] + rem / (win * win);
            const int64_t s = (int64_t)p * g.ncell +
                              ((int64_t)wrap_index(cz, g.nz) * g.ny + wrap_index(cy, g.ny)) * g.nx +
                              wrap_index(cx, g.nx);
            const double ux = S.ux[s];
            if (ux > VACANT_TEST) continue;
            const double u[3] = {ux, S.uy[s], S.uz[s]};
            double d[3];
            lat_sep(cx, cy, cz, p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) {
                const double rr = sqrt(r2);
                double df, dphi, phi;
                fp_phi(rr, T, df, dphi, phi);
                const double fpj = real_is_f32 ? (double)((const float *)S.fp)[s] : ((const double *)S.fp)[s];
                const double sc_ = ((fpr + fpj) * df + dphi) / rr;
                fx += sc_ * d[0];
                fy += sc_ * d[1];
                fz += sc_ * d[2];
                ep += phi;  // lattice partner has no other record of this pair's energy
            }
        }
        for_runaway_neighbours(x, r, lane, 64, g.rc2, S, sc, g, [&](int o, const double *d, double r2) {
            const double rr = sqrt(r2);
            double df, dphi, phi;
            fp_phi(rr, T, df, dphi, phi);
            const double sc_ = ((fpr + S.r_fp[o]) * df + dphi) / rr;
            fx += sc_ * d[0];
            fy += sc_ * d[1];
            fz += sc_ * d[2];
            ep += 0.5 * phi;
        });
        fx = wave_sum64(fx);
        fy = wave_sum64(fy);
        fz = wave_sum64(fz);
        ep = wave_sum64(ep);
        if (lane == 0) {
            S.r_fx[r] = fx;
            S.r_fy[r] = fy;
            S.r_fz[r] = fz;
            if (energy) S.r_e[2 * r + 1] = ep;
        }
    }
}

// kick != 0: the force pass already applied the second half-kick with the lattice
// part of F; add the run-away part's kick here and record |v|^2 for the step statistics.
template <typename Real>
__global__ void k_affected_force(State S, Scratch sc, Geom g, Tables<double> T, int kick, double kf) {
    int na = sc.cnt->n_affected;
    na = na < sc.affected_cap ? na : (int)sc.affected_cap;
    const double hk = kick ? 0.5 * sc.scal[0] * kf : 0.0;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < na; q += gridDim.x * blockDim.x) {
        const int64_t s = sc.affected[q];
        const int p = s >= g.ncell ? 1 : 0;
        const int64_t c = s - p * g.ncell;
        const int cxj = (int)(c % g.nx), cyj = (int)((c / g.nx) % g.ny), czj = (int)(c / ((int64_t)g.nx * g.ny));
        const double u[3] = {S.ux[s], S.uy[s], S.uz[s]};
        Real *fxa = (Real *)S.fx;
        Real *fya = (Real *)S.fy;
        Real *fza = (Real *)S.fz;
        const double fpj = (double)((const Real *)S.fp)[s];
        double xj[3];
        site_pos(cxj, cyj, czj, p, g.a, xj);
        for (int k = 0; k < 3; ++k) xj[k] = wrap_coord(xj[k] + u[k], g.L[k]);
        double ax = 0.0, ay = 0.0, az = 0.0;
        for_runaway_neighbours(xj, -1, 0, 1, g.pre2, S, sc, g, [&](int o, const double *, double) {
            const double x[3] = {S.r_x[o], S.r_y[o], S.r_z[o]};
            int cc[3];
            const int cj[3] = {cxj, cyj, czj};
            const int nn[3] = {g.nx, g.ny, g.nz};
            for (int k = 0; k < 3; ++k) {
                const int lo = window_lo(x[k] * g.inv_a, g.reach);
                cc[k] = lo + wrap_index(cj[k] - lo, nn[k]);
                if (cc[k] - lo >= g.win) return;
            }
            double d[3];  // x_j - x_o
            lat_sep(cc[0], cc[1], cc[2], p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) {
                const double rr = sqrt(r2);
                double df, dphi, phi;
                fp_phi(rr, T, df, dphi, phi);
                const double sc_ = ((fpj + S.r_fp[o]) * df + dphi) / rr;
                ax -= sc_ * d[0];  // separation from j to the run-away is -d
                ay -= sc_ * d[1];
                az -= sc_ * d[2];
            }
        });
        fxa[s] = (Real)((double)fxa[s] + ax);
        fya[s] = (Real)((double)fya[s] + ay);
        fza[s] = (Real)((double)fza[s] + az);
        if (kick) {
            const double vx = S.vx[s] + hk * ax, vy = S.vy[s] + hk * ay, vz = S.vz[s] + hk * az;
            S.vx[s] = vx;
            S.vy[s] = vy;
            S.vz[s] = vz;
            sc.aff_v2[q] = vx * vx + vy * vy + vz * vz;
        }
        sc.mark[s >> 5] = 0u;  // every bit of a touched word belongs to an affected site
    }
}

// Ascending sort of the affected list (site indices), so every later pass over it and
// the sums taken along it run in a fixed order.  Single work-group; sorts in place in
// global memory (capacity is a power of two) when the list exceeds the LDS buffer.
constexpr int SORT32_LDS_MAX = 8192;
__global__ __launch_bounds__(SORT_THREADS) void k_sort_affected(Scratch sc) {
    __shared__ int32_t sh[SORT32_LDS_MAX];
    int n = sc.cnt->n_affected;
    n = n < sc.affected_cap ? n : (int)sc.affected_cap;
    if (n <= 1) return;
    int P = 1;
    while (P < n) P <<= 1;
    const bool in_lds = P <= SORT32_LDS_MAX;
    int32_t *A = in_lds ? sh : sc.affected;
    for (int i = threadIdx.x; i < P; i += SORT_THREADS) {
        if (in_lds)
            sh[i] = i < n ? sc.affected[i] : INT32_MAX;
        else if (i >= n)
            sc.affected[i] = INT32_MAX;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += SORT_THREADS) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int32_t a = A[i], b = A[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        A[i] = b;
                        A[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (in_lds)
        for (int i = threadIdx.x; i < n; i += SORT_THREADS) sc.affected[i] = sh[i];
}

// ---------------------------------------------------------------------------
// launchers

static Tables<double> t64_of(misa_lattice *h) {
    Tables<double> T;
    T.f = h->t64.f;
    T.force = h->t64.force;
    T.phi = h->t64.phi;
    T.emb = h->t64.emb;
    T.fm = h->t64.fm;
    T.em = h->t64.em;
    return T;
}

static Tables<float> t32_of(misa_lattice *h) {
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    return T;
}

hipError_t launch_rehash(misa_lattice *h) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_sort, dim3(1), dim3(SORT_THREADS), 0, st, h->sc.sortbuf, 0, h->sc.cnt, h->rcap, h->sc.l_id,
                       nullptr, nullptr, nullptr, h->g);
    hipLaunchKernelGGL(k_claim, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_settle, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, h->S, h->sc);
    return hipGetLastError();
}

hipError_t launch_runaway_build(misa_lattice *h) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_sort, dim3(1), dim3(SORT_THREADS), 0, st, h->sc.sortbuf, 1, h->sc.cnt, h->rcap, nullptr,
                       h->S.r_x, h->S.r_y, h->S.r_z, h->g);
    hipLaunchKernelGGL(k_hash_insert, dim3(SMALL_GRID), dim3(256), 0, st, h->sc);
    return hipGetLastError();
}

hipError_t launch_runaway_rho(misa_lattice *h) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_runaway_rho, dim3(SMALL_GRID), dim3(64 * RUNAWAY_WAVES_PER_BLOCK), 0, st, h->S, h->sc,
                       h->g, t64_of(h));
    hipLaunchKernelGGL(k_sort_affected, dim3(1), dim3(SORT_THREADS), 0, st, h->sc);
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_affected_rho<float>, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g, t64_of(h),
                           t32_of(h));
    else
        hipLaunchKernelGGL(k_affected_rho<double>, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g,
                           t64_of(h), t64_of(h));
    return hipGetLastError();
}

hipError_t launch_runaway_force(misa_lattice *h, bool energy, bool kick) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_runaway_force, dim3(SMALL_GRID), dim3(64 * RUNAWAY_WAVES_PER_BLOCK), 0, st, h->S, h->sc,
                       h->g, t64_of(h), h->precision == MISA_FP32 ? 1 : 0, energy ? 1 : 0);
    const double kf = ACC_UNIT / h->mass;
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_affected_force<float>, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g,
                           t64_of(h), kick ? 1 : 0, kf);
    else
        hipLaunchKernelGGL(k_affected_force<double>, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g,
                           t64_of(h), kick ? 1 : 0, kf);
    return hipGetLastError();
}

hipError_t launch_runaway_clear(misa_lattice *h) {
    hipLaunchKernelGGL(k_hash_clear, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->sc);
    return hipGetLastError();
}

}  // namespace misa
