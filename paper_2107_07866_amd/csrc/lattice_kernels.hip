// Lattice-array kernels: the array-array part of the EAM evaluation
// (Algorithm 1, first loop; Sec. 2.2 steps 1-5) as a full-neighbour gather.
//
// Every work-group stages a TX x TY x TZ brick of cells of both sublattices,
// plus a periodic halo of HALO cells, in LDS (the paper's ghost region, D6,
// realised as a wrap at tile load).  One lane owns one site; the loop over the
// Neighbor Offset Index is wave-uniform, so the table look-ups of a wave fall in
// one narrow band of r (the same locality the paper gains by moving the offset
// loop outermost, Sec. 4.1).  Each pair is evaluated from both ends, so no
// write conflicts arise and no colouring or atomics are needed.
#include "misa_internal.h"

#include <type_traits>

namespace misa {


__device__ __forceinline__ int wrapg(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Load the tile (interior + halo) of both sublattices into LDS.  w_src (may
// be null) supplies the fourth component (F' for the force pass).
template <typename Real>
__device__ __forceinline__ float load_tile(Q4<Real> *__restrict__ tile, const double *__restrict__ ux,
                                           const double *__restrict__ uy, const double *__restrict__ uz,
                                           const Real *__restrict__ w_src, const Geom &g, int bx, int by,
                                           int bz) {
    float m = 0.0f;  // largest |u|^2 of the occupied sites this lane loaded
    for (int e = threadIdx.x; e < TILE_SITES; e += TILE_THREADS) {
        int lx = e % PX;
        int r = e / PX;
        int ly = r % PY;
        r /= PY;
        int lz = r % PZ;
        int p = r / PZ;
        int gx = wrapg(bx + lx, g.nx), gy = wrapg(by + ly, g.ny), gz = wrapg(bz + lz, g.nz);
        int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        Q4<Real> q;
        q.x = (Real)ux[idx];
        q.y = (Real)uy[idx];
        q.z = (Real)uz[idx];
        q.w = w_src ? w_src[idx] : (Real)0;
        tile[e] = q;
        if (q.x < (Real)VACANT_TEST) m = fmaxf(m, (float)(q.x * q.x + q.y * q.y + q.z * q.z));
    }
    return m;
}

// Stencil length for this tile (after the tile is in LDS): entries kin .. K - 1 lie
// beyond rc + 2 u_cut, so when every occupied site of the tile and its halo has
// |u|^2 < u_cut2 they hold no pair within rc and are skipped.
__device__ __forceinline__ int tile_length(float m, unsigned *slot, int K, int kin, float u_cut2) {
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));  // |u|^2 >= 0: integer order = float order
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(__uint_as_float(*slot) < u_cut2 ? kin : K);
}

// rho_i = sum_j f(r_ij) over the stencil, then F'(rho_i) (Sec. 2.2 steps 1-2).
template <typename Real>
__global__ __launch_bounds__(TILE_THREADS) void k_rho_tile(
    const double *__restrict__ ux, const double *__restrict__ uy, const double *__restrict__ uz,
    Real *__restrict__ rho, Real *__restrict__ fp, const StencilEntry<Real> *__restrict__ st, int K, int kin,
    float u_cut2, const Q4<Real> *__restrict__ ftab, TabMeta<Real> fm, const Q4<Real> *__restrict__ etab,
    TabMeta<Real> em, Geom g, uint32_t *__restrict__ range_viol, const NearTab *__restrict__ nt) {
    __shared__ Q4<Real> tile[TILE_SITES];
    __shared__ unsigned umax;
    const int tid = tile_of_block(blockIdx.x, g);
    if (tid >= g.ntiles) return;  // whole work-group leaves together
    if (threadIdx.x == 0) umax = 0u;
    const int tx = tid % g.ntx;
    const int tyz = tid / g.ntx;
    const int ty = tyz % g.nty;
    const int tz = tyz / g.nty;
    const float m = load_tile<Real>(tile, ux, uy, uz, nullptr, g, tx * TX - HALO, ty * TY - HALO, tz * TZ - HALO);
    __syncthreads();
    K = tile_length(m, &umax, K, kin, u_cut2);

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform parity: stencil entries are fetched with scalar loads
    const int p = __builtin_amdgcn_readfirstlane(w / TZ);
    const int lz = w % TZ, lx = lane % TX, ly = lane / TX;
    const int gx = tx * TX + lx, gy = ty * TY + ly, gz = tz * TZ + lz;
    if (gx >= g.nx || gy >= g.ny || gz >= g.nz) return;
    const int me = ((p * PZ + lz + HALO) * PY + ly + HALO) * PX + lx + HALO;
    const Q4<Real> ui = tile[me];
    const Real rc2 = (Real)g.rc2;
    const StencilEntry<Real> *sp = st + p * KMAX;
    const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
    Real acc = 0;
    // Branch-free and unrolled: every candidate gathers its (clamped) record and an
    // out-of-range pair is dropped by a select, so the L2 gathers of several
    // candidates are in flight together.
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        const StencilEntry<Real> e = sp[k];
        const Q4<Real> uj = tile[me + e.lds];
        const Real dx = (uj.x - ui.x) + e.ox;
        const Real dy = (uj.y - ui.y) + e.oy;
        const Real dz = (uj.z - ui.z) + e.oz;
        const Real r2 = dx * dx + dy * dy + dz * dz;
        bool in = r2 < rc2;
        if (std::is_same<Real, float>::value && fabsf((float)r2 - (float)rc2) < RC_BAND_Q)  // float64 re-decision
            in = pair_in_rc64(ux, uy, uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny, g.nz, g.ncell, nt->rc2);
        int s;
        Real t;
        seg_index(pair_r<Real>(in ? r2 : rc2), fm, s, t);
        const Q4<Real> c = ftab[s];
        const Real v = ((c.w * t + c.z) * t + c.y) * t + c.x;
        acc += in ? v : (Real)0;
    }
    Real fpv = 0;
    bool beyond = false;
    if (ui.x > (Real)VACANT_TEST) {
        acc = 0;
    } else {
        Real Fv;
        fpv = emb_eval<Real>(acc, etab, em, Fv, beyond);
    }
    rho[idx] = acc;
    fp[idx] = fpv;
    if (beyond) atomicAdd(range_viol, 1u);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The second half-kick of velocity Verlet fused into the force pass: v += (dt/2) C F / m
// as soon as F_i is known, plus per-tile {max |v|^2, sum |v|^2} over the atoms no
// run-away atom touches (those get their run-away terms, kick and statistics later).
struct KickArgs {
    double *vx, *vy, *vz;
    const uint32_t *mark;
    const double *scal;  // scal[0] = dt of the current step
    double *part_kick;
    double kf;           // C / m
};

// f'(r) and phi'(r) of segment s at t.  Float64 gathers the dense 48-byte record
// (three 16-byte loads); float32 the two 16-byte records.
template <typename Real>
__device__ __forceinline__ void force_rec(const Tables<Real> &T, int s, Real t, Real &dfr, Real &dph) {
    const Q4<Real> a = T.force[2 * s];
    const Q4<Real> b = T.force[2 * s + 1];
    dfr = (a.z * t + a.y) * t + a.x;
    dph = (b.y * t + b.x) * t + a.w;
}
template <>
__device__ __forceinline__ void force_rec<double>(const Tables<double> &T, int s, double t, double &dfr, double &dph) {
    const double2 *r = reinterpret_cast<const double2 *>(T.force6) + 3 * s;
    const double2 q0 = r[0], q1 = r[1], q2 = r[2];  // {f'0, f'1}, {f'2, phi'0}, {phi'1, phi'2}
    dfr = (q1.x * t + q0.y) * t + q0.x;
    dph = (q2.y * t + q2.x) * t + q1.y;
}

// F_i = sum_j [(F'_i + F'_j) f'(r) + phi'(r)] (x_j - x_i) / r   (Eq. eam_force_ij)
// With kEnergy: per-tile partial sums of F(rho_i) and 1/2 sum_j phi(r_ij).
template <typename Real, bool kEnergy, bool kKick>
__global__ __launch_bounds__(TILE_THREADS) void k_force_tile(
    const double *__restrict__ ux, const double *__restrict__ uy, const double *__restrict__ uz,
    const Real *__restrict__ fp, const Real *__restrict__ rho, Real *__restrict__ fx, Real *__restrict__ fy,
    Real *__restrict__ fz, const StencilEntry<Real> *__restrict__ st, int K, int kin, float u_cut2, Tables<Real> T,
    Geom g, double *__restrict__ part, KickArgs kick, const NearTab *__restrict__ nt) {
    __shared__ Q4<Real> tile[TILE_SITES];
    __shared__ double red[4][TILE_THREADS / 64];
    __shared__ unsigned umax;
    const int tid = tile_of_block(blockIdx.x, g);
    if (tid >= g.ntiles) return;
    if (threadIdx.x == 0) umax = 0u;
    const int tx = tid % g.ntx;
    const int tyz = tid / g.ntx;
    const int ty = tyz % g.nty;
    const int tz = tyz / g.nty;
    const float m = load_tile<Real>(tile, ux, uy, uz, fp, g, tx * TX - HALO, ty * TY - HALO, tz * TZ - HALO);
    __syncthreads();
    K = tile_length(m, &umax, K, kin, u_cut2);

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform parity: stencil entries are fetched with scalar loads
    const int p = __builtin_amdgcn_readfirstlane(w / TZ);
    const int lz = w % TZ, lx = lane % TX, ly = lane / TX;
    const int gx = tx * TX + lx, gy = ty * TY + ly, gz = tz * TZ + lz;
    const bool active = gx < g.nx && gy < g.ny && gz < g.nz;
    const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
    double e_emb = 0.0, e_pair = 0.0, kvm = 0.0, kvs = 0.0;
    double v0x = 0.0, v0y = 0.0, v0z = 0.0;
    uint32_t mw = 0u;
    if (kKick && active) {  // issued now, consumed after the pair loop
        v0x = kick.vx[idx];
        v0y = kick.vy[idx];
        v0z = kick.vz[idx];
        mw = kick.mark[idx >> 5];
    }
    if (active) {
        const int me = ((p * PZ + lz + HALO) * PY + ly + HALO) * PX + lx + HALO;
        const Q4<Real> ui = tile[me];
        const Real rc2 = (Real)g.rc2;
        const StencilEntry<Real> *sp = st + p * KMAX;
        Real ax = 0, ay = 0, az = 0, ep = 0;
        // branch-free and unrolled, as in the rho pass
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            const StencilEntry<Real> e = sp[k];
            const Q4<Real> uj = tile[me + e.lds];
            const Real dx = (uj.x - ui.x) + e.ox;
            const Real dy = (uj.y - ui.y) + e.oy;
            const Real dz = (uj.z - ui.z) + e.oz;
            const Real r2 = dx * dx + dy * dy + dz * dz;
            bool in = r2 < rc2;
            if (std::is_same<Real, float>::value && fabsf((float)r2 - (float)rc2) < RC_BAND_Q)  // float64 re-decision
                in = pair_in_rc64(ux, uy, uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny, g.nz, g.ncell,
                                  nt->rc2);
            Real r, rinv;
            pair_r_rinv<Real>(in ? r2 : rc2, r, rinv);
            int s;
            Real t;
            seg_index(r, T.fm, s, t);
            Real dfr, dph;  // f'(r), phi'(r)
            force_rec<Real>(T, s, t, dfr, dph);
            const Real sc = in ? ((ui.w + uj.w) * dfr + dph) * rinv : (Real)0;
            ax += sc * dx;
            ay += sc * dy;
            az += sc * dz;
            if (kEnergy) {
                const Q4<Real> c = T.phi[s];
                const Real v = ((c.w * t + c.z) * t + c.y) * t + c.x;
                ep += in ? v : (Real)0;
            }
        }
        const bool vac = ui.x > (Real)VACANT_TEST;
        if (vac) ax = ay = az = 0;
        fx[idx] = ax;
        fy[idx] = ay;
        fz[idx] = az;
        if (kKick && !vac) {
            const double hk = 0.5 * kick.scal[0] * kick.kf;
            const double vx = v0x + hk * (double)ax;
            const double vy = v0y + hk * (double)ay;
            const double vz = v0z + hk * (double)az;
            kick.vx[idx] = vx;
            kick.vy[idx] = vy;
            kick.vz[idx] = vz;
            if (!((mw >> (idx & 31)) & 1u)) {
                kvm = vx * vx + vy * vy + vz * vz;
                kvs = kvm;
            }
        }
        if (kEnergy && !vac) {
            Real Fv;
            bool beyond = false;
            emb_eval<Real>(rho[idx], T.emb, T.em, Fv, beyond);
            e_emb = (double)Fv;
            e_pair = 0.5 * (double)ep;
        }
    }
    if (kEnergy || kKick) {
        if (kEnergy) {
            e_emb = wave_sum(e_emb);
            e_pair = wave_sum(e_pair);
        }
        if (kKick) {
            for (int o = 32; o >= 1; o >>= 1) kvm = fmax(kvm, __shfl_xor(kvm, o, 64));
            kvs = wave_sum(kvs);
        }
        if (lane == 0) {
            red[0][w] = e_emb;
            red[1][w] = e_pair;
            red[2][w] = kvm;
            red[3][w] = kvs;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0, m2 = 0.0, s3 = 0.0;
            for (int q = 0; q < TILE_THREADS / 64; ++q) {
                s0 += red[0][q];
                s1 += red[1][q];
                m2 = fmax(m2, red[2][q]);
                s3 += red[3][q];
            }
            if (kEnergy) {
                part[2 * tid] = s0;
                part[2 * tid + 1] = s1;
            }
            if (kKick) {
                kick.part_kick[2 * tid] = m2;
                kick.part_kick[2 * tid + 1] = s3;
            }
        }
    }
}

template <typename Real>
static Tables<Real> tables_of(const DevTables<Real> &t) {
    Tables<Real> T;
    T.force6 = t.force6;
    T.f = t.f;
    T.force = t.force;
    T.phi = t.phi;
    T.emb = t.emb;
    T.fm = t.fm;
    T.em = t.em;
    return T;
}

template <typename Real>
static hipError_t rho_impl(misa_lattice *h, const StencilEntry<Real> *st, const DevTables<Real> &t) {
    const Geom &g = h->g;
    hipLaunchKernelGGL(k_rho_tile<Real>, dim3(g.ntiles_pad), dim3(TILE_THREADS), 0, h->stream, h->S.ux, h->S.uy,
                       h->S.uz, (Real *)h->S.rho, (Real *)h->S.fp, st, h->K, h->K_in, h->u_cut2, t.f, t.fm, t.emb,
                       t.em, g, &h->sc.cnt->range_viol, near_args(h, false));
    return hipGetLastError();
}

hipError_t launch_rho(misa_lattice *h) {
    if (h->use_mlp) return half_mlp_path(h) ? launch_rho_half_mlp(h) : launch_rho_mlp(h);
    if (half_path(h)) return launch_rho_half(h);
    if (lds_path(h)) return launch_rho_lds(h);
    if (h->precision == MISA_FP32) return rho_impl<float>(h, h->st32, h->t32);
    if (lds64_path(h)) return launch_rho_lds64(h);
    return rho_impl<double>(h, h->st64, h->t64);
}

template <typename Real, bool kEnergy, bool kKick>
static void force_variant(misa_lattice *h, const StencilEntry<Real> *st, const Tables<Real> &T, const KickArgs &ka) {
    const Geom &g = h->g;
    hipLaunchKernelGGL((k_force_tile<Real, kEnergy, kKick>), dim3(g.ntiles_pad), dim3(TILE_THREADS), 0, h->stream,
                       h->S.ux, h->S.uy, h->S.uz, (const Real *)h->S.fp, (const Real *)h->S.rho, (Real *)h->S.fx,
                       (Real *)h->S.fy, (Real *)h->S.fz, st, h->K, h->K_in, h->u_cut2, T, g, h->sc.part, ka,
                       near_args(h, false));
}

template <typename Real>
static hipError_t force_impl(misa_lattice *h, bool energy, bool kick, const StencilEntry<Real> *st,
                             const DevTables<Real> &t) {
    const Tables<Real> T = tables_of(t);
    const KickArgs ka{h->S.vx, h->S.vy, h->S.vz, h->sc.mark, h->sc.scal, h->sc.part_kick, ACC_UNIT / h->mass};
    if (energy && kick) force_variant<Real, true, true>(h, st, T, ka);
    else if (energy) force_variant<Real, true, false>(h, st, T, ka);
    else if (kick) force_variant<Real, false, true>(h, st, T, ka);
    else force_variant<Real, false, false>(h, st, T, ka);
    return hipGetLastError();
}

// Every table form but the learned one and the half-stencil schedule kicks inside the force pass.
bool fused_kick(const misa_lattice *h) { return !h->use_mlp && !half_path(h); }

bool force_on_tiles2(const misa_lattice *h) {
    return lds_path(h) || half_mlp_path(h) || lds64f_path(h);
}

hipError_t launch_force(misa_lattice *h, bool energy, bool kick) {
    if (half_path(h)) return kick ? hipErrorInvalidValue : launch_force_half(h, energy);
    if (lds_path(h)) return launch_force_lds(h, energy, kick);
    if (h->use_mlp) {
        if (kick) return hipErrorInvalidValue;  // the learned form keeps the separate final kick
        return half_mlp_path(h) ? launch_force_half_mlp(h, energy) : launch_force_mlp(h, energy);
    }
    if (h->precision == MISA_FP32) return force_impl<float>(h, energy, kick, h->st32, h->t32);
    if (lds64f_path(h)) return launch_force_lds64(h, energy, kick);
    return force_impl<double>(h, energy, kick, h->st64, h->t64);
}

// Final energy sums: per-tile partials, per-run-away terms and the pair-energy
// corrections of the affected list, fixed order.
__device__ __forceinline__ void energy_reduce_body(const double *__restrict__ part, int ntiles,
                                                        const double *__restrict__ r_e,
                                                        const double *__restrict__ aff_e, int64_t aff_cap,
                                                        const Counters *__restrict__ cnt,
                                                        double *__restrict__ scal, double *__restrict__ out) {
    __shared__ double red[2][1024 / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += 1024) {
        s0 += part[2 * i];
        s1 += part[2 * i + 1];
    }
    const int nr = cnt->n_run;
    for (int i = threadIdx.x; i < nr; i += 1024) {
        s0 += r_e[2 * i];
        s1 += r_e[2 * i + 1];
    }
    const int na = cnt->n_affected < aff_cap ? cnt->n_affected : (int)aff_cap;
    for (int i = threadIdx.x; i < na; i += 1024) s1 += aff_e[i];
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = s0;
        red[1][w] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < 1024 / 64; ++q) {
            a += red[0][q];
            b += red[1][q];
        }
        scal[4] = a;
        scal[5] = b;
        if (out) {
            out[0] = a;
            out[1] = b;
        }
    }
}

__global__ __launch_bounds__(1024) void k_energy_reduce(const double *__restrict__ part, int ntiles,
                                                        const double *__restrict__ r_e,
                                                        const double *__restrict__ aff_e, int64_t aff_cap,
                                                        const Counters *__restrict__ cnt,
                                                        double *__restrict__ scal, double *__restrict__ out) {
    energy_reduce_body(part, ntiles, r_e, aff_e, aff_cap, cnt, scal, out);
}

__global__ __launch_bounds__(1024) void kb_energy_reduce(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    energy_reduce_body(B.sc.part, B.g.ntiles2, B.S.r_e, B.sc.aff_e, B.sc.affected_cap, B.sc.cnt, B.sc.scal, nullptr);
}


hipError_t launchb_energy_reduce(hipStream_t st, const BoxRef *boxes, int nbox) {
    hipLaunchKernelGGL(kb_energy_reduce, dim3(1, nbox), dim3(1024), 0, st, boxes);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(misa_lattice *h, double *energies_dev) {
    // per-tile partials of the force pass used (8 x 8 x 8 tiles or the generic tiles)
    const int nparts = force_on_tiles2(h) ? h->g.ntiles2 : h->g.ntiles;
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(1024), 0, h->stream, h->sc.part, nparts, h->S.r_e,
                       h->sc.aff_e, h->sc.affected_cap, h->sc.cnt, h->sc.scal, energies_dev);
    return hipGetLastError();
}

}  // namespace misa
