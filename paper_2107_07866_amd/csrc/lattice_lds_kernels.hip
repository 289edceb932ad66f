// Persistent float32 lattice kernels (rho pass and force pass).
//
// Same gather as the generic tile kernels, reorganised for the table look-ups
// that dominate the pair loop (the same pressure the paper meets on the 64 KiB
// local store, Sec. 4.1): each work-group copies, once, the window of the f /
// phi coefficient records that pairs of slotted atoms can reach
// (r >= nearest-site distance - 2 delta) into LDS, then loops over 8 x 8 x 8-cell
// tiles, each staged with its periodic halo.  Work-groups are sized to one per
// compute unit; tiles are dealt out so every XCD sweeps one contiguous block of
// tiles (halo re-reads stay in that XCD's L2).
//
// The pair loop is branch-free and unrolled: every stencil candidate runs the
// full arithmetic and out-of-range pairs are dropped by a select, so the LDS
// reads of several offsets are in flight together instead of one dependent
// chain per offset.  Table indices are clamped into the window: a slotted atom
// is within delta of its site, so an in-range pair can only fall below the
// window after a run-away capacity overflow (reported on its own).
#include "misa_internal.h"

namespace misa {

__device__ __forceinline__ int wrap2(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Tile handled by work-group b on its it-th iteration, or -1 when done.
__device__ __forceinline__ int persistent_tile(int b, int it, int grid, const Geom &g) {
    const int per = g.ntiles2_pad >> 3;         // tiles per XCD
    const int j = (b >> 3) + it * (grid >> 3);  // position inside this XCD's block of tiles
    if (j >= per) return -1;
    return (b & 7) * per + j;
}

__device__ __forceinline__ void load_tile2(Q4<float> *__restrict__ tile, const double *__restrict__ ux,
                                           const double *__restrict__ uy, const double *__restrict__ uz,
                                           const float *__restrict__ w_src, const Geom &g, int tid) {
    const int tx = tid % g.nt2[0];
    const int tyz = tid / g.nt2[0];
    const int ty = tyz % g.nt2[1];
    const int tz = tyz / g.nt2[1];
    const int bx = tx * T2X - HALO, by = ty * T2Y - HALO, bz = tz * T2Z - HALO;
    for (int e = threadIdx.x; e < TILE2_SITES; e += TILE2_THREADS) {
        const int lx = e % P2X;
        int r = e / P2X;
        const int ly = r % P2Y;
        r /= P2Y;
        const int lz = r % P2Z;
        const int p = r / P2Z;
        const int gx = wrap2(bx + lx, g.nx), gy = wrap2(by + ly, g.ny), gz = wrap2(bz + lz, g.nz);
        const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        Q4<float> q;
        q.x = (float)ux[idx];
        q.y = (float)uy[idx];
        q.z = (float)uz[idx];
        q.w = w_src ? w_src[idx] : 0.0f;
        tile[e] = q;
    }
}

// Local segment index and offset t for pp = (r - x0) / h - k0 (the window starts
// at segment k0).  With kNodeCut the last node sits at the cut-off and the window
// ends with a zero record at local index nwin: pairs at or beyond the cut-off read
// zeros, so no separate cut-off select is needed.
template <bool kNodeCut>
__device__ __forceinline__ int win_seg(float pp, int nwin, float &t) {
    const float top = kNodeCut ? (float)nwin : (float)(nwin - 1);
    t = __builtin_amdgcn_fractf(pp);
    return (int)__builtin_amdgcn_fmed3f(pp, 0.0f, top);
}

template <bool kNodeCut>
__global__ __launch_bounds__(TILE2_THREADS) void k_rho_lds(
    const double *__restrict__ ux, const double *__restrict__ uy, const double *__restrict__ uz,
    float *__restrict__ rho, float *__restrict__ fp, const StencilEntry<float> *__restrict__ st, int K,
    const Q4<float> *__restrict__ fwin, int k0, int nwin, TabMeta<float> fm, const Q4<float> *__restrict__ etab,
    TabMeta<float> em, Geom g, uint32_t *__restrict__ range_viol) {
    __shared__ Q4<float> tile[TILE2_SITES];
    __shared__ float4 ftab[LDS_TAB_SEGS];
    for (int e = threadIdx.x; e < nwin; e += TILE2_THREADS) {
        const Q4<float> c = fwin[e];
        ftab[e] = make_float4(c.x, c.y, c.z, c.w);
    }
    if (kNodeCut && threadIdx.x == 0) ftab[nwin] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform: the stencil entries below become scalar loads
    const int p = __builtin_amdgcn_readfirstlane(w / T2Z);
    const int lz = w % T2Z, lx = lane % T2X, ly = lane / T2X;
    const StencilEntry<float> *sp = st + p * KMAX;
    const float rc2 = (float)g.rc2;
    const float pc = -fm.x0 * fm.inv_h - (float)k0;  // pp = (r - x0) / h - k0
    for (int it = 0;; ++it) {
        const int tid = persistent_tile(blockIdx.x, it, gridDim.x, g);
        if (tid < 0) break;
        if (tid >= g.ntiles2) continue;  // uniform across the work-group
        __syncthreads();                 // previous tile fully consumed (and table copied)
        load_tile2(tile, ux, uy, uz, nullptr, g, tid);
        __syncthreads();
        const int tx = tid % g.nt2[0];
        const int tyz = tid / g.nt2[0];
        const int gx = tx * T2X + lx, gy = (tyz % g.nt2[1]) * T2Y + ly, gz = (tyz / g.nt2[1]) * T2Z + lz;
        if (gx >= g.nx || gy >= g.ny || gz >= g.nz) continue;
        const int me = ((p * P2Z + lz + HALO) * P2Y + ly + HALO) * P2X + lx + HALO;
        const Q4<float> ui = tile[me];
        float acc = 0.0f;
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            const StencilEntry<float> e = sp[k];
            const Q4<float> uj = tile[me + e.lds];
            const float dx = (uj.x - ui.x) + e.ox;
            const float dy = (uj.y - ui.y) + e.oy;
            const float dz = (uj.z - ui.z) + e.oz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            float t;
            const int s = win_seg<kNodeCut>(__builtin_amdgcn_sqrtf(r2) * fm.inv_h + pc, nwin, t);
            const float4 c = ftab[s];
            const float v = ((c.w * t + c.z) * t + c.y) * t + c.x;
            acc += (kNodeCut || r2 < rc2) ? v : 0.0f;
        }
        const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        float fpv = 0.0f;
        bool beyond = false;
        if (ui.x > (float)VACANT_TEST) {
            acc = 0.0f;
        } else if (acc > em.x_last) {
            beyond = true;
            fpv = em.d_last;
        } else {
            const float q = (acc - em.x0) * em.inv_h;
            int kk = (int)q;
            kk = kk < em.nseg - 1 ? kk : em.nseg - 1;
            kk = kk > 0 ? kk : 0;
            const float t = q - (float)kk;
            const Q4<float> d = etab[2 * kk + 1];
            fpv = (d.z * t + d.y) * t + d.x;
        }
        rho[idx] = acc;
        fp[idx] = fpv;
        if (beyond) atomicAdd(range_viol, 1u);
    }
}

__device__ __forceinline__ double wave_sum_l(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool kEnergy, bool kNodeCut>
__global__ __launch_bounds__(TILE2_THREADS) void k_force_lds(
    const double *__restrict__ ux, const double *__restrict__ uy, const double *__restrict__ uz,
    const float *__restrict__ fp, const float *__restrict__ rho, float *__restrict__ fx, float *__restrict__ fy,
    float *__restrict__ fz, const StencilEntry<float> *__restrict__ st, int K, const FRec32 *__restrict__ fwin,
    int k0, int nwin, Tables<float> T, Geom g, double *__restrict__ part) {
    __shared__ Q4<float> tile[TILE2_SITES];
    __shared__ float4 fab[LDS_TAB_SEGS];  // {f'0, f'1, f'2, phi'0} per segment
    __shared__ float2 fcc[LDS_TAB_SEGS];  // {phi'1, phi'2}
    __shared__ double red[2][TILE2_THREADS / 64];
    for (int e = threadIdx.x; e < nwin; e += TILE2_THREADS) {
        const FRec32 c = fwin[e];
        fab[e] = make_float4(c.a.x, c.a.y, c.b.x, c.b.y);
        fcc[e] = c.c;
    }
    if (kNodeCut && threadIdx.x == 0) {
        fab[nwin] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        fcc[nwin] = make_float2(0.0f, 0.0f);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w / T2Z);
    const int lz = w % T2Z, lx = lane % T2X, ly = lane / T2X;
    const StencilEntry<float> *sp = st + p * KMAX;
    const float rc2 = (float)g.rc2;
    const float inv_h = T.fm.inv_h;
    const float pc = -T.fm.x0 * T.fm.inv_h - (float)k0;  // pp = (r - x0) / h - k0
    const int nlast = T.fm.nseg - 1;
    for (int it = 0;; ++it) {
        const int tid = persistent_tile(blockIdx.x, it, gridDim.x, g);
        if (tid < 0) break;
        if (tid >= g.ntiles2) continue;
        __syncthreads();
        load_tile2(tile, ux, uy, uz, fp, g, tid);
        __syncthreads();
        const int tx = tid % g.nt2[0];
        const int tyz = tid / g.nt2[0];
        const int gx = tx * T2X + lx, gy = (tyz % g.nt2[1]) * T2Y + ly, gz = (tyz / g.nt2[1]) * T2Z + lz;
        const bool active = gx < g.nx && gy < g.ny && gz < g.nz;
        double e_emb = 0.0, e_pair = 0.0;
        if (active) {
            const int me = ((p * P2Z + lz + HALO) * P2Y + ly + HALO) * P2X + lx + HALO;
            const Q4<float> ui = tile[me];
            float ax = 0.0f, ay = 0.0f, az = 0.0f, ep = 0.0f;
#pragma unroll 4
            for (int k = 0; k < K; ++k) {
                const StencilEntry<float> e = sp[k];
                const Q4<float> uj = tile[me + e.lds];
                const float dx = (uj.x - ui.x) + e.ox;
                const float dy = (uj.y - ui.y) + e.oy;
                const float dz = (uj.z - ui.z) + e.oz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                float t;
                const int s = win_seg<kNodeCut>((r2 * rinv) * inv_h + pc, nwin, t);
                const float4 a = fab[s];
                const float2 c = fcc[s];
                const float dfr = (a.z * t + a.y) * t + a.x;  // f'(r)
                const float dph = (c.y * t + c.x) * t + a.w;  // phi'(r)
                float sc = ((ui.w + uj.w) * dfr + dph) * rinv;
                if (!kNodeCut) sc = r2 < rc2 ? sc : 0.0f;
                ax += sc * dx;
                ay += sc * dy;
                az += sc * dz;
                if (kEnergy) {
                    const int sg = min(s + k0, nlast);
                    const Q4<float> cp = T.phi[sg];
                    const float v = ((cp.w * t + cp.z) * t + cp.y) * t + cp.x;
                    ep += (kNodeCut ? s < nwin : r2 < rc2) ? v : 0.0f;  // same pair set as the force
                }
            }
            const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
            const bool vac = ui.x > (float)VACANT_TEST;
            if (vac) ax = ay = az = 0.0f;
            fx[idx] = ax;
            fy[idx] = ay;
            fz[idx] = az;
            if (kEnergy && !vac) {
                const float rr = rho[idx];
                float Fv;
                if (rr > T.em.x_last) {
                    Fv = T.em.y_last + T.em.d_last * (rr - T.em.x_last);
                } else {
                    const float q = (rr - T.em.x0) * T.em.inv_h;
                    int kk = (int)q;
                    kk = kk < T.em.nseg - 1 ? kk : T.em.nseg - 1;
                    kk = kk > 0 ? kk : 0;
                    const float t = q - (float)kk;
                    const Q4<float> c = T.emb[2 * kk];
                    Fv = ((c.w * t + c.z) * t + c.y) * t + c.x;
                }
                e_emb = (double)Fv;
                e_pair = 0.5 * (double)ep;
            }
        }
        if (kEnergy) {
            e_emb = wave_sum_l(e_emb);
            e_pair = wave_sum_l(e_pair);
            if (lane == 0) {
                red[0][w] = e_emb;
                red[1][w] = e_pair;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double s0 = 0.0, s1 = 0.0;
                for (int q = 0; q < TILE2_THREADS / 64; ++q) {
                    s0 += red[0][q];
                    s1 += red[1][q];
                }
                part[2 * tid] = s0;
                part[2 * tid + 1] = s1;
            }
        }
    }
}

bool lds_path(const misa_lattice *h) {
    return h->precision == MISA_FP32 && h->lds32.usable && h->persistent_grid > 0;
}

hipError_t launch_rho_lds(misa_lattice *h) {
    const Geom &g = h->g;
    auto kern = h->lds32.node_cut ? k_rho_lds<true> : k_rho_lds<false>;
    hipLaunchKernelGGL(kern, dim3(h->persistent_grid), dim3(TILE2_THREADS), 0, h->stream, h->S.ux, h->S.uy, h->S.uz,
                       (float *)h->S.rho, (float *)h->S.fp, h->st32p, h->K, h->lds32.f, h->lds32.k0, h->lds32.nwin,
                       h->t32.fm, h->t32.emb, h->t32.em, g, &h->sc.cnt->range_viol);
    return hipGetLastError();
}

hipError_t launch_force_lds(misa_lattice *h, bool energy) {
    const Geom &g = h->g;
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    const bool nc = h->lds32.node_cut;
    auto kern = energy ? (nc ? k_force_lds<true, true> : k_force_lds<true, false>)
                       : (nc ? k_force_lds<false, true> : k_force_lds<false, false>);
    hipLaunchKernelGGL(kern, dim3(h->persistent_grid), dim3(TILE2_THREADS), 0, h->stream, h->S.ux, h->S.uy, h->S.uz,
                       (const float *)h->S.fp, (const float *)h->S.rho, (float *)h->S.fx, (float *)h->S.fy,
                       (float *)h->S.fz, h->st32p, h->K, h->lds32.force, h->lds32.k0, h->lds32.nwin, T, g,
                       h->sc.part);
    return hipGetLastError();
}

}  // namespace misa
