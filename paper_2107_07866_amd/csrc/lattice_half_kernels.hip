// Half-stencil float32 lattice passes: every unordered pair is evaluated once.
//
// Newton's third law halves the pair work of the rho and force passes (the
// paper's Sec. 4.2); the price is a write to the partner atom as well, which two
// threads may share.  The paper avoids those write conflicts by colouring
// z blocks of the domain red and blue and running one colour after the other.
// The GPU form here:
//  * Pair ownership.  The pair (i, j = i + o) belongs to i when the lattice-id
//    offset o points into the forward half space: dZ > 0, or dZ = 0 and dY > 0,
//    or dZ = dY = 0 and dX > 0.  The odd-parity stencil is the negated even one,
//    so exactly one end of every pair owns it.
//  * Footprint.  An 8 x 8 x 8-cell tile stages the sites its forward pairs reach:
//    x and y from -2 to +10 cells, z from 0 to +10, both sublattices.  Terms for
//    footprint sites accumulate in LDS and are added to HBM when the tile ends.
//  * Colours.  Tiles are 2-coloured per axis (8 colours, one launch each).  Two
//    tiles of one colour are 16 cells apart, so their footprints never overlap
//    and the write-back is a plain read-add-write; the colours run in a fixed
//    order.
//  * Phases.  Inside a tile a wave serves one z plane of one parity.  The stencil
//    is split into 6 phases by (dZ, parity change); within a phase every wave
//    writes a different (plane, parity) of the footprint, so no two waves touch
//    one LDS word, and barriers separate the phases.  The partner terms are
//    therefore plain LDS read-add-writes (LDS float atomics measured ~20x slower
//    than reads).  Within a wave they stay in program order: two stencil
//    entries' partner addresses may coincide for all the compiler knows, and
//    the LDS serves one wave's accesses in order.  Every site receives its
//    terms in a fixed order: results are bit-reproducible run to run.
// The pair arithmetic (displacement form, q = r^2 table window in LDS, zero
// record at the cut-off) is that of the full-gather persistent kernels.
#include "misa_internal.h"

#include <type_traits>

#include "mlp_wave.h"

namespace misa {

constexpr int HF_THREADS = TILE2_THREADS;                              // 1024: one lane per interior site
constexpr int HF_PER_LANE = (HT_SITES + HF_THREADS - 1) / HF_THREADS;  // footprint sites per lane

__device__ __forceinline__ int hf_wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Tile of colour c (bits: x, y, z parity of the tile coordinates) for item it of
// work-group b, dealt so that every XCD sweeps one contiguous block of items.
struct ColourTiles {
    int nt0, nt1, nt2;  // tiles per axis (even)
    int colour;
    int nitems, nitems_pad;
    __device__ __forceinline__ int next(int b, int &it, int grid) const {
        const int per = nitems_pad >> 3;
        for (;; ++it) {
            const int j = (b >> 3) + it * (grid >> 3);
            if (j >= per) return -1;
            const int id = (b & 7) * per + j;
            if (id < nitems) return id;
        }
    }
    // item -> tile coordinates and tile id (the id the energy partials use)
    __device__ __forceinline__ int tile(int item, int &tx, int &ty, int &tz) const {
        const int hx = nt0 >> 1, hy = nt1 >> 1;
        const int ix = item % hx, r = item / hx;
        const int iy = r % hy, iz = r / hy;
        tx = 2 * ix + (colour & 1);
        ty = 2 * iy + ((colour >> 1) & 1);
        tz = 2 * iz + ((colour >> 2) & 1);
        return (tz * nt1 + ty) * nt0 + tx;
    }
};

// Footprint entry e -> (lx, ly, lz, p) of the staged block and its storage index.
__device__ __forceinline__ int64_t hf_site(int e, int tx, int ty, int tz, const Geom &g) {
    const int lx = e % HFX;
    int r = e / HFX;
    const int ly = r % HFY;
    r /= HFY;
    const int lz = r % HFZ;
    const int p = r / HFZ;
    const int gx = hf_wrap(tx * T2X - HALO + lx, g.nx);
    const int gy = hf_wrap(ty * T2Y - HALO + ly, g.ny);
    const int gz = hf_wrap(tz * T2Z + lz, g.nz);
    return (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
}

// One lane's share of a footprint in registers: displacements (and F') to stage,
// and the values the write-back adds to (NOUT arrays: rho, or F_x, F_y, F_z).
// Same-colour footprints are disjoint and earlier colours have finished, so those
// values cannot change during the launch and are fetched a tile ahead.
template <int NOUT, int NT = HF_THREADS>
struct HfRegs {
    static constexpr int PER = (HT_SITES + NT - 1) / NT;  // footprint sites per lane
    double x[PER], y[PER], z[PER];
    float w[PER];
    float old[NOUT > 0 ? NOUT : 1][PER];
};

template <int NOUT, int NT = HF_THREADS>
__device__ __forceinline__ void hf_fetch(HfRegs<NOUT, NT> &R, const State &S, float *const *out, bool with_fp,
                                         int tx, int ty, int tz, const Geom &g) {
#pragma unroll
    for (int j = 0; j < HfRegs<NOUT, NT>::PER; ++j) {
        const int e = threadIdx.x + j * NT;
        if (e < HT_SITES) {
            const int64_t idx = hf_site(e, tx, ty, tz, g);
            R.x[j] = S.ux[idx];
            R.y[j] = S.uy[idx];
            R.z[j] = S.uz[idx];
            R.w[j] = with_fp ? ((const float *)S.fp)[idx] : 0.0f;
#pragma unroll
            for (int c = 0; c < NOUT; ++c) R.old[c][j] = out[c][idx];
        }
    }
}

// Stores the staged displacements, zeroes the accumulators (NACC floats per
// footprint site), returns max |u|^2 of the occupied sites this lane stored.
template <int NACC, int NOUT, int NT = HF_THREADS>
__device__ __forceinline__ float hf_store(Q4<float> *__restrict__ tile, float *__restrict__ acc,
                                          const HfRegs<NOUT, NT> &R) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < HfRegs<NOUT, NT>::PER; ++j) {
        const int e = threadIdx.x + j * NT;
        if (e < HT_SITES) {
            Q4<float> q;
            q.x = (float)R.x[j];
            q.y = (float)R.y[j];
            q.z = (float)R.z[j];
            q.w = R.w[j];
            tile[e] = q;
#pragma unroll
            for (int c = 0; c < NACC; ++c) acc[NACC * e + c] = 0.0f;  // NACC floats per footprint site
            if (q.x < (float)VACANT_TEST) m = fmaxf(m, q.x * q.x + q.y * q.y + q.z * q.z);
        }
    }
    return m;
}

// Whether every occupied site of the footprint has |u|^2 below u_cut2 (then the
// entries beyond rc of each phase cannot hold a pair within rc).  Contains the
// barrier after which the staged tile is visible.
// safe: bit k set when entry k (this lane's threshold: thr) holds no pair near rc
// in this tile, so its cut-off decision needs no band test (NearTab).
__device__ __forceinline__ bool hf_near_sites(float m, unsigned *slot, unsigned *other, float u_cut2, float thr,
                                              uint64_t &safe) {
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));
    __syncthreads();
    const float umax2 = __uint_as_float(*slot);
    if (threadIdx.x == 0) *other = 0u;
    safe = __ballot(umax2 < thr);
    return __builtin_amdgcn_readfirstlane(umax2 < u_cut2 ? 1 : 0) != 0;
}
__device__ __forceinline__ bool hf_near_sites(float m, unsigned *slot, unsigned *other, float u_cut2) {
    uint64_t safe;
    return hf_near_sites(m, slot, other, u_cut2, -1.0f, safe);
}

// First entry of [k0, k1) that needs the band test: the safe entries of a phase
// are a prefix of it (nearest first).
__device__ __forceinline__ int hf_klo(uint64_t safe, int k0, int k1) {
    const uint64_t in = k1 - k0 >= 64 ? ~0ull : ((1ull << (k1 - k0)) - 1ull);
    return __builtin_amdgcn_readfirstlane(k0 + __popcll((safe >> k0) & in));
}

template <bool kNodeCut>
__device__ __forceinline__ int hf_seg(float pp, int nwin, float &t) {
    const float top = kNodeCut ? (float)nwin : (float)(nwin - 1);
    t = __builtin_amdgcn_fractf(pp);
    return (int)__builtin_amdgcn_fmed3f(pp, 0.0f, top);
}

// ---------------------------------------------------------------------------
// rho: rho_i and rho_j += f(r) for every owned pair; one launch per colour.
template <bool kNodeCut>
__global__ __launch_bounds__(HF_THREADS) void k_rho_half(ColourTiles ct, State S, Geom g,
                                                         const StencilEntry<float> *__restrict__ hst,
                                                         const int32_t *__restrict__ hmeta,
                                                         const Q4<float> *__restrict__ fwin, float inv_hq,
                                                         float pcq, int nwin, float rc2, float u_cut2,
                                                         const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[HT_SITES];
    __shared__ float acc[HT_SITES];
    __shared__ float4 ftab[HALF_TAB_SEGS];
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    for (int e = threadIdx.x; e < nwin; e += HF_THREADS) {
        const Q4<float> c = fwin[e];
        ftab[e] = make_float4(c.x, c.y, c.z, c.w);
    }
    if (kNodeCut && threadIdx.x == 0) ftab[nwin] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w / T2Z);
    const int lz = w % T2Z, lx = lane % T2X, ly = lane / T2X;
    // wave-uniform parity: the stencil entries and phase bounds become scalar loads
    const StencilEntry<float> *sp = hst + p * KMAX;
    const int32_t *meta = hmeta + p * HALF_META;
    const int me = ((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO;
    const float thr = nt->thr2[p][lane];
    float *const out[1] = {(float *)S.rho};
    int it = 0;
    int item = ct.next(blockIdx.x, it, gridDim.x);
    HfRegs<1> R;
    float old[1][HF_PER_LANE];
    int tx, ty, tz;
    if (item >= 0) {
        ct.tile(item, tx, ty, tz);
        hf_fetch<1>(R, S, out, false, tx, ty, tz, g);
    }
    while (item >= 0) {
        ct.tile(item, tx, ty, tz);
        __syncthreads();  // previous tile written back (and the table copied)
        const float m = hf_store<1>(tile, acc, R);
#pragma unroll
        for (int jj = 0; jj < HF_PER_LANE; ++jj) old[0][jj] = R.old[0][jj];
        uint64_t safe;
        const bool near =
            hf_near_sites(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], u_cut2, thr, safe);
        ++it;
        const int nxt = ct.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            int nx_, ny_, nz_;
            ct.tile(nxt, nx_, ny_, nz_);
            hf_fetch<1>(R, S, out, false, nx_, ny_, nz_, g);  // in flight during this tile
        }
        const Q4<float> ui = tile[me];
        const int gx = tx * T2X + lx, gy = ty * T2Y + ly, gz = tz * T2Z + lz;
        const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        float ai = 0.0f;
        // f(r) of entry k to both ends; kCheck: the cut-off decision of a pair within
        // the band around rc^2 is taken again in float64
        auto term = [&](int k, auto check) {
            const StencilEntry<float> e = sp[k];
            const int j = me + e.lds;
            const Q4<float> uj = tile[j];
            const float dx = (uj.x - ui.x) + e.ox;
            const float dy = (uj.y - ui.y) + e.oy;
            const float dz = (uj.z - ui.z) + e.oz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            float t;
            const int s = hf_seg<kNodeCut>(r2 * inv_hq + pcq, nwin, t);
            const float4 c = ftab[s];
            const float vr = ((c.w * t + c.z) * t + c.y) * t + c.x;
            float v = (kNodeCut || r2 < rc2) ? vr : 0.0f;
            if (decltype(check)::value && fabsf(r2 - rc2) < RC_BAND_Q) {
                const bool in = pair_in_rc64(S.ux, S.uy, S.uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny,
                                             g.nz, g.ncell, nt->rc2);
                if (kNodeCut && s >= nwin) {  // past the window's last node (rc) in float32: f there
                    const float4 cl = ftab[nwin - 1];
                    v = in ? cl.x + cl.y + cl.z + cl.w : 0.0f;
                } else {
                    v = in ? vr : 0.0f;
                }
            }
            ai += v;
            acc[j] += v;  // no other wave writes this plane in this phase
        };
        for (int q = 0; q < HALF_PHASES; ++q) {
            const int k0 = __builtin_amdgcn_readfirstlane(meta[q]);
            const int k1 = __builtin_amdgcn_readfirstlane(near ? k0 + meta[8 + q] : meta[q + 1]);
            const int kl = hf_klo(safe, k0, k1);
#pragma unroll 4
            for (int k = k0; k < kl; ++k) term(k, std::false_type{});
#pragma unroll 4
            for (int k = kl; k < k1; ++k) term(k, std::true_type{});
            __syncthreads();  // the next phase's waves write other planes of the footprint
        }
        acc[me] += ai;  // the site's own pairs, after every partner term
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < HF_PER_LANE; ++jj) {
            const int e = threadIdx.x + jj * HF_THREADS;
            if (e < HT_SITES) out[0][hf_site(e, tx, ty, tz, g)] = old[0][jj] + acc[e];
        }
        item = nxt;
    }
}

// F'(rho) of every site after the last colour (empty slots: rho = F' = 0).
__global__ void k_embed_half(State S, Geom g, Tables<float> T, unsigned *range_viol) {
    float *rho = (float *)S.rho;
    float *fp = (float *)S.fp;
    unsigned nb = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.nsites;
         s += (int64_t)gridDim.x * blockDim.x) {
        const float r = rho[s];
        float d;
        if (S.atom[s] == VACANT_ID) {
            rho[s] = 0.0f;
            d = 0.0f;
        } else if (r > T.em.x_last) {
            d = T.em.d_last;
            ++nb;
        } else {
            const float q = (r - T.em.x0) * T.em.inv_h;
            int kk = (int)q;
            kk = kk < T.em.nseg - 1 ? kk : T.em.nseg - 1;
            kk = kk > 0 ? kk : 0;
            const float t = q - (float)kk;
            const Q4<float> c = T.emb[2 * kk + 1];
            d = (c.z * t + c.y) * t + c.x;
        }
        fp[s] = d;
    }
    if (nb) atomicAdd(range_viol, nb);
}

// ---------------------------------------------------------------------------
// force: F_i += s d, F_j -= s d for every owned pair (s = (F'_i + F'_j) f'/r + phi'/r);
// with kEnergy also the per-tile sums of F(rho_i) and of phi over the owned pairs.
template <bool kEnergy, bool kNodeCut>
__global__ __launch_bounds__(HF_THREADS) void k_force_half(ColourTiles ct, State S, Geom g,
                                                           const StencilEntry<float> *__restrict__ hst,
                                                           const int32_t *__restrict__ hmeta,
                                                           const FRec32 *__restrict__ fwin, float inv_hq,
                                                           float pcq, int nwin, Tables<float> T, float rc2,
                                                           float u_cut2, double *__restrict__ part, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[HT_SITES];
    __shared__ float4 acc[HT_SITES];       // {F_x, F_y, F_z, -} per footprint site: one 16-byte read-add-write
    __shared__ float4 fab[HALF_TAB_SEGS];  // {f'0, f'1, f'2, phi'0} per segment
    __shared__ float2 fcc[HALF_TAB_SEGS];  // {phi'1, phi'2}
    __shared__ unsigned umax_slot[2];
    __shared__ double red[2][HF_THREADS / 64];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    for (int e = threadIdx.x; e < nwin; e += HF_THREADS) {
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
    // wave-uniform parity: the stencil entries and phase bounds become scalar loads
    const StencilEntry<float> *sp = hst + p * KMAX;
    const int32_t *meta = hmeta + p * HALF_META;
    const int me = ((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO;
    const float thr = nt->thr2[p][lane];
    const int nlast = T.fm.nseg - 1;
    float *const out[3] = {(float *)S.fx, (float *)S.fy, (float *)S.fz};
    int it = 0;
    int item = ct.next(blockIdx.x, it, gridDim.x);
    HfRegs<3> R;
    float old[3][HF_PER_LANE];
    int tx, ty, tz;
    if (item >= 0) {
        ct.tile(item, tx, ty, tz);
        hf_fetch<3>(R, S, out, true, tx, ty, tz, g);
    }
    while (item >= 0) {
        const int tid = ct.tile(item, tx, ty, tz);
        __syncthreads();
        const float m = hf_store<4>(tile, (float *)acc, R);
#pragma unroll
        for (int jj = 0; jj < HF_PER_LANE; ++jj) {
            old[0][jj] = R.old[0][jj];
            old[1][jj] = R.old[1][jj];
            old[2][jj] = R.old[2][jj];
        }
        uint64_t safe;
        const bool near =
            hf_near_sites(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], u_cut2, thr, safe);
        ++it;
        const int nxt = ct.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            int nx_, ny_, nz_;
            ct.tile(nxt, nx_, ny_, nz_);
            hf_fetch<3>(R, S, out, true, nx_, ny_, nz_, g);
        }
        const Q4<float> ui = tile[me];
        const int gx = tx * T2X + lx, gy = ty * T2Y + ly, gz = tz * T2Z + lz;
        const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        float ax = 0.0f, ay = 0.0f, az = 0.0f, ep = 0.0f;
        // the pair term of entry k to both ends; kCheck: the cut-off decision of a pair
        // within the band around rc^2 is taken again in float64
        auto term = [&](int k, auto check) {
            const StencilEntry<float> e = sp[k];
            const int j = me + e.lds;
            const Q4<float> uj = tile[j];
            const float dx = (uj.x - ui.x) + e.ox;
            const float dy = (uj.y - ui.y) + e.oy;
            const float dz = (uj.z - ui.z) + e.oz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            float t;
            const int s = hf_seg<kNodeCut>(r2 * inv_hq + pcq, nwin, t);
            const float4 a = fab[s];
            const float2 c = fcc[s];
            float gf = (a.z * t + a.y) * t + a.x;  // f'(r) / r
            float gp = (c.y * t + c.x) * t + a.w;  // phi'(r) / r
            bool in = kNodeCut ? s < nwin : r2 < rc2;
            if (decltype(check)::value && fabsf(r2 - rc2) < RC_BAND_Q) {
                in = pair_in_rc64(S.ux, S.uy, S.uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny, g.nz,
                                  g.ncell, nt->rc2);
                if (kNodeCut && s >= nwin) {  // past the window's last node (rc) in float32: the records there
                    const float4 al = fab[nwin - 1];
                    const float2 cl = fcc[nwin - 1];
                    gf = al.x + al.y + al.z;
                    gp = al.w + cl.x + cl.y;
                }
                gf = in ? gf : 0.0f;
                gp = in ? gp : 0.0f;
            }
            float sc = (ui.w + uj.w) * gf + gp;
            if (!kNodeCut) sc = in ? sc : 0.0f;
            const float px = sc * dx, py = sc * dy, pz = sc * dz;
            ax += px;
            ay += py;
            az += pz;
            float4 aj = acc[j];  // no other wave writes this plane in this phase
            aj.x -= px;
            aj.y -= py;
            aj.z -= pz;
            acc[j] = aj;
            if (kEnergy) {
                const float pr = (__builtin_amdgcn_sqrtf(r2) - T.fm.x0) * T.fm.inv_h;
                const int sg = max(0, min((int)pr, nlast));
                const float tr = pr - (float)sg;
                const Q4<float> cp = T.phi[sg];
                const float v = ((cp.w * tr + cp.z) * tr + cp.y) * tr + cp.x;
                ep += in ? v : 0.0f;
            }
        };
        for (int q = 0; q < HALF_PHASES; ++q) {
            const int k0 = __builtin_amdgcn_readfirstlane(meta[q]);
            const int k1 = __builtin_amdgcn_readfirstlane(near ? k0 + meta[8 + q] : meta[q + 1]);
            const int kl = hf_klo(safe, k0, k1);
#pragma unroll 4
            for (int k = k0; k < kl; ++k) term(k, std::false_type{});
#pragma unroll 4
            for (int k = kl; k < k1; ++k) term(k, std::true_type{});
            __syncthreads();
        }
        {
            float4 am = acc[me];
            am.x += ax;
            am.y += ay;
            am.z += az;
            acc[me] = am;
        }
        if (kEnergy) {
            double e_emb = 0.0, e_pair = 0.0;
            if (ui.x < (float)VACANT_TEST) {
                const int gx = tx * T2X + lx, gy = ty * T2Y + ly, gz = tz * T2Z + lz;
                const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
                const float rr = ((const float *)S.rho)[idx];
                float Fv;
                if (rr > T.em.x_last) {
                    Fv = T.em.y_last + T.em.d_last * (rr - T.em.x_last);
                } else {
                    const float qq = (rr - T.em.x0) * T.em.inv_h;
                    int kk = (int)qq;
                    kk = kk < T.em.nseg - 1 ? kk : T.em.nseg - 1;
                    kk = kk > 0 ? kk : 0;
                    const float tt = qq - (float)kk;
                    const Q4<float> c = T.emb[2 * kk];
                    Fv = ((c.w * tt + c.z) * tt + c.y) * tt + c.x;
                }
                e_emb = (double)Fv;
                e_pair = (double)ep;
            }
            for (int o = 32; o >= 1; o >>= 1) {
                e_emb += __shfl_xor(e_emb, o, 64);
                e_pair += __shfl_xor(e_pair, o, 64);
            }
            if (lane == 0) {
                red[0][w] = e_emb;
                red[1][w] = e_pair;
            }
        }
        __syncthreads();
        if (kEnergy && threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < HF_THREADS / 64; ++q) {
                s0 += red[0][q];
                s1 += red[1][q];
            }
            part[2 * tid] = s0;
            part[2 * tid + 1] = s1;
        }
#pragma unroll
        for (int jj = 0; jj < HF_PER_LANE; ++jj) {
            const int e = threadIdx.x + jj * HF_THREADS;
            if (e < HT_SITES) {
                const int64_t idx = hf_site(e, tx, ty, tz, g);
                const float4 a = acc[e];
                out[0][idx] = old[0][jj] + a.x;
                out[1][idx] = old[1][jj] + a.y;
                out[2][idx] = old[2][jj] + a.z;
            }
        }
        item = nxt;
    }
}

// ---------------------------------------------------------------------------
// The learned form on the half stencil: the f and phi networks (matrix cores, whole
// waves) replace the table window, each owned pair is evaluated once; pairs outside
// a network's range take the float32 tables from memory, as in the gather form.

struct HalfNets {
    MlpNet f, phi, emb;
    const uint16_t *w2f, *w2p, *w2e;  // W2 of each network as bfloat16 bits
};

// 512 lanes per tile: wave w serves z plane w of both parities, one after the other
// inside each phase (the 16 (plane, parity) write targets of a phase stay disjoint),
// which leaves each lane the registers of two networks with their tangents.
constexpr int HFM_THREADS = 512;

// The rho pass evaluates the f network with its tangent and keeps f'(r) of every owned
// pair in dfbuf (entry k of the site with storage index i at k nsites + i), so that the
// force pass only runs the phi network.
__global__ __launch_bounds__(HFM_THREADS) void k_rho_half_mlp(ColourTiles ct, State S, Geom g,
                                                              const StencilEntry<float> *__restrict__ hst,
                                                              const int32_t *__restrict__ hmeta, HalfNets N,
                                                              Tables<float> T, float rc2, float u_cut2,
                                                              float *__restrict__ dfbuf, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[HT_SITES];
    __shared__ float acc[HT_SITES];
    __shared__ MlpLds Lf;
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    fill_lds(Lf, N.f.p);
    bf16x4_t Af[4];
    load_a(Af, N.w2f);
    const MlpNet nf = N.f;
    const int lz = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = lane % T2X, ly = lane / T2X;
    float *const out[1] = {(float *)S.rho};
    int it = 0;
    int item = ct.next(blockIdx.x, it, gridDim.x);
    while (item >= 0) {
        int tx, ty, tz;
        ct.tile(item, tx, ty, tz);
        __syncthreads();  // previous tile written back (and the network constants stored)
        float m;
        {
            // fetched when needed: the networks cost ~100x the fetch latency per tile,
            // and the registers a prefetch would hold go to the networks
            HfRegs<0, HFM_THREADS> R;
            hf_fetch<0, HFM_THREADS>(R, S, nullptr, false, tx, ty, tz, g);
            m = hf_store<1, 0, HFM_THREADS>(tile, acc, R);
        }
        const bool near = hf_near_sites(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], u_cut2);
        ++it;
        const int nxt = ct.next(blockIdx.x, it, gridDim.x);
        float ai[2] = {0.0f, 0.0f};
        const float kfd = nf.y_scale * nf.s;
        const int64_t cell = ((int64_t)(tz * T2Z + lz) * g.ny + (ty * T2Y + ly)) * g.nx + (tx * T2X + lx);
        for (int q = 0; q < HALF_PHASES; ++q) {
            for (int p = 0; p < 2; ++p) {
                const StencilEntry<float> *sp = hst + p * KMAX;
                const int32_t *meta = hmeta + p * HALF_META;
                const int me = ((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO;
                const int64_t idx = (int64_t)p * g.ncell + cell;
                const Q4<float> ui = tile[me];
                const int k0 = __builtin_amdgcn_readfirstlane(meta[q]);
                const int k1 = __builtin_amdgcn_readfirstlane(near ? k0 + meta[8 + q] : meta[q + 1]);
                for (int k = k0; k < k1; ++k) {
                    const StencilEntry<float> e = sp[k];
                    const int j = me + e.lds;
                    const Q4<float> uj = tile[j];
                    const float dx = (uj.x - ui.x) + e.ox;
                    const float dy = (uj.y - ui.y) + e.oy;
                    const float dz = (uj.z - ui.z) + e.oz;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float r = __builtin_amdgcn_sqrtf(r2);
                    float y, dyt;
                    mlp_wave<true>(Lf, Af, net_t(nf, r), y, dyt);  // every lane: the whole wave runs it
                    float v = 0.0f, dfr = 0.0f;
                    bool in = r2 < rc2;
                    if (fabsf(r2 - rc2) < RC_BAND_Q)  // cut-off decided again in float64 (NearTab)
                        in = pair_in_rc64(S.ux, S.uy, S.uz, idx, tx * T2X + lx, ty * T2Y + ly, tz * T2Z + lz, p,
                                          nt->st[p][k], g.nx, g.ny, g.nz, g.ncell, nt->rc2);
                    if (in) {
                        v = nf.y_shift + nf.y_scale * y;
                        dfr = kfd * dyt;
                        if (!mlp_serves(nf, r)) {
                            int sg;
                            float t;
                            seg32(r, T.fm, sg, t);
                            const Q4<float> c = T.f[sg];
                            v = ((c.w * t + c.z) * t + c.y) * t + c.x;
                            const Q4<float> a = T.force[2 * sg];
                            dfr = (a.z * t + a.y) * t + a.x;
                        }
                    }
                    dfbuf[(int64_t)k * g.nsites + idx] = dfr;
                    ai[p] += v;
                    acc[j] += v;  // no other wave writes this (plane, parity) in this phase
                }
            }
            __syncthreads();
        }
        for (int p = 0; p < 2; ++p) acc[((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO] += ai[p];
        __syncthreads();
        // same-colour footprints are disjoint and earlier colours are done: a plain read-add-write
        for (int e = threadIdx.x; e < HT_SITES; e += HFM_THREADS) {
            const int64_t idx = hf_site(e, tx, ty, tz, g);
            out[0][idx] += acc[e];
        }
        item = nxt;
    }
}

// F'(rho) from the embedding network after the last colour, 64 sites per wave (the
// whole wave evaluates; lanes past the end compute on a clamped site and store nothing).
__global__ __launch_bounds__(256) void k_embed_half_mlp(State S, Geom g, HalfNets N, Tables<float> T,
                                                        unsigned *range_viol) {
    __shared__ MlpLds Le;
    fill_lds(Le, N.emb.p);
    bf16x4_t Ae[4];
    load_a(Ae, N.w2e);
    __syncthreads();
    const MlpNet ne = N.emb;
    float *rho = (float *)S.rho;
    float *fp = (float *)S.fp;
    unsigned nb = 0;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = wave0; base < g.nsites; base += stride) {
        const int64_t s = base + (threadIdx.x & 63);
        const bool valid = s < g.nsites;
        const int64_t sc = valid ? s : g.nsites - 1;
        const bool vac = S.atom[sc] == VACANT_ID;
        const float r = vac ? 0.0f : rho[sc];
        float ye, de;
        mlp_wave<true>(Le, Ae, net_t(ne, r), ye, de);
        float d = ne.y_scale * ne.s * de;
        bool beyond = false;
        if (!mlp_serves(ne, r)) {
            float Fv;
            d = emb_tab(r, T, Fv, beyond);
        }
        if (vac) d = 0.0f;
        if (valid) {
            if (vac) rho[s] = 0.0f;
            fp[s] = d;
            nb += beyond ? 1u : 0u;
        }
    }
    if (nb) atomicAdd(range_viol, nb);
}

// F_i += s d, F_j -= s d for every owned pair with s from the f and phi networks;
// with kEnergy the per-tile sums of F(rho_i) (embedding network) and phi.
template <bool kEnergy>
__global__ __launch_bounds__(HFM_THREADS) void k_force_half_mlp(ColourTiles ct, State S, Geom g,
                                                                const StencilEntry<float> *__restrict__ hst,
                                                                const int32_t *__restrict__ hmeta, HalfNets N,
                                                                Tables<float> T, float rc2, float u_cut2,
                                                                double *__restrict__ part,
                                                                const float *__restrict__ dfbuf, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[HT_SITES];
    __shared__ float4 acc[HT_SITES];
    __shared__ MlpLds Lp, Le;
    __shared__ unsigned umax_slot[2];
    __shared__ double red[2][HFM_THREADS / 64];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    fill_lds(Lp, N.phi.p);
    if (kEnergy) fill_lds(Le, N.emb.p);
    bf16x4_t Ap[4];
    load_a(Ap, N.w2p);
    const MlpNet np = N.phi;
    const float kp = np.y_scale * np.s;
    const int lz = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = lane % T2X, ly = lane / T2X;
    float *const out[3] = {(float *)S.fx, (float *)S.fy, (float *)S.fz};
    int it = 0;
    int item = ct.next(blockIdx.x, it, gridDim.x);
    while (item >= 0) {
        int tx, ty, tz;
        const int tid = ct.tile(item, tx, ty, tz);
        __syncthreads();
        float m;
        {
            HfRegs<0, HFM_THREADS> R;  // fetched when needed, as in the rho pass
            hf_fetch<0, HFM_THREADS>(R, S, nullptr, true, tx, ty, tz, g);
            m = hf_store<4, 0, HFM_THREADS>(tile, (float *)acc, R);
        }
        const bool near = hf_near_sites(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], u_cut2);
        ++it;
        const int nxt = ct.next(blockIdx.x, it, gridDim.x);
        // the two parities one after the other: all phases of parity 0, its own sums,
        // then parity 1 (a phase's (plane, parity) write targets are disjoint either way)
        float epp[2] = {0.0f, 0.0f};
        const int64_t cell = ((int64_t)(tz * T2Z + lz) * g.ny + (ty * T2Y + ly)) * g.nx + (tx * T2X + lx);
#pragma unroll 1
        for (int p = 0; p < 2; ++p) {
            const StencilEntry<float> *sp = hst + p * KMAX;
            const int32_t *meta = hmeta + p * HALF_META;
            const int me = ((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO;
            const int64_t idx = (int64_t)p * g.ncell + cell;
            const Q4<float> ui = tile[me];
            float ax = 0.0f, ay = 0.0f, az = 0.0f, ep = 0.0f;
            for (int q = 0; q < HALF_PHASES; ++q) {
                const int k0 = __builtin_amdgcn_readfirstlane(meta[q]);
                const int k1 = __builtin_amdgcn_readfirstlane(near ? k0 + meta[8 + q] : meta[q + 1]);
                for (int k = k0; k < k1; ++k) {
                    const StencilEntry<float> e = sp[k];
                    const int j = me + e.lds;
                    const Q4<float> uj = tile[j];
                    const float dx = (uj.x - ui.x) + e.ox;
                    const float dy = (uj.y - ui.y) + e.oy;
                    const float dz = (uj.z - ui.z) + e.oz;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * rinv;
                    const float dfr = dfbuf[(int64_t)k * g.nsites + idx];  // f'(r) from the rho pass
                    float yp, dp;
                    mlp_wave<true>(Lp, Ap, net_t(np, r), yp, dp);  // every lane: the whole wave runs it
                    float px = 0.0f, py = 0.0f, pz = 0.0f;
                    bool in = r2 < rc2;
                    if (fabsf(r2 - rc2) < RC_BAND_Q)  // cut-off decided again in float64 (NearTab)
                        in = pair_in_rc64(S.ux, S.uy, S.uz, idx, tx * T2X + lx, ty * T2Y + ly, tz * T2Z + lz, p,
                                          nt->st[p][k], g.nx, g.ny, g.nz, g.ncell, nt->rc2);
                    if (in) {
                        float dph = kp * dp, ph = np.y_shift + np.y_scale * yp;
                        if (!mlp_serves(np, r)) {
                            int sg;
                            float t;
                            seg32(r, T.fm, sg, t);
                            const Q4<float> a = T.force[2 * sg], b = T.force[2 * sg + 1];
                            dph = (b.y * t + b.x) * t + a.w;
                            const Q4<float> c = T.phi[sg];
                            ph = ((c.w * t + c.z) * t + c.y) * t + c.x;
                        }
                        const float sc = ((ui.w + uj.w) * dfr + dph) * rinv;
                        px = sc * dx;
                        py = sc * dy;
                        pz = sc * dz;
                        if (kEnergy) ep += ph;
                    }
                    ax += px;
                    ay += py;
                    az += pz;
                    float4 aj = acc[j];  // no other wave writes this (plane, parity) in this phase
                    aj.x -= px;
                    aj.y -= py;
                    aj.z -= pz;
                    acc[j] = aj;
                }
                __syncthreads();
            }
            float4 am = acc[me];
            am.x += ax;
            am.y += ay;
            am.z += az;
            acc[me] = am;
            epp[p] = ep;
            __syncthreads();  // before the other parity's partner writes reach these sites
        }
        if (kEnergy) {
            bf16x4_t Ae[4];
            load_a(Ae, N.w2e);
            double e_emb = 0.0, e_pair = 0.0;
            for (int p = 0; p < 2; ++p) {
                const int me = ((p * HFZ + lz) * HFY + ly + HALO) * HFX + lx + HALO;
                const bool vac = tile[me].x > (float)VACANT_TEST;
                const int gx = tx * T2X + lx, gy = ty * T2Y + ly, gz = tz * T2Z + lz;
                const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
                const float rr = vac ? 0.0f : ((const float *)S.rho)[idx];
                float ye, unused;
                mlp_wave<false>(Le, Ae, net_t(N.emb, rr), ye, unused);
                float Fv = N.emb.y_shift + N.emb.y_scale * ye;
                if (!mlp_serves(N.emb, rr)) {
                    bool beyond = false;
                    emb_tab(rr, T, Fv, beyond);
                }
                e_emb += vac ? 0.0 : (double)Fv;
                e_pair += vac ? 0.0 : (double)epp[p];
            }
            for (int o = 32; o >= 1; o >>= 1) {
                e_emb += __shfl_xor(e_emb, o, 64);
                e_pair += __shfl_xor(e_pair, o, 64);
            }
            if (lane == 0) {
                red[0][lz] = e_emb;
                red[1][lz] = e_pair;
            }
        }
        __syncthreads();
        if (kEnergy && threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < HFM_THREADS / 64; ++w) {
                s0 += red[0][w];
                s1 += red[1][w];
            }
            part[2 * tid] = s0;
            part[2 * tid + 1] = s1;
        }
        // same-colour footprints are disjoint and earlier colours are done: a plain read-add-write
        for (int e = threadIdx.x; e < HT_SITES; e += HFM_THREADS) {
            const int64_t idx = hf_site(e, tx, ty, tz, g);
            const float4 a = acc[e];
            out[0][idx] += a.x;
            out[1][idx] += a.y;
            out[2][idx] += a.z;
        }
        item = nxt;
    }
}

__global__ void k_zero_f32(float *__restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0f;
}

bool half_path(const misa_lattice *h) {
    return h->pair_schedule == MISA_PAIRS_HALF && lds_path(h) && h->lds32h.usable && h->half_fits;
}

bool half_mlp_path(const misa_lattice *h) {
    return h->pair_schedule == MISA_PAIRS_HALF && h->use_mlp && h->half_fits && h->persistent_grid > 0 &&
           h->pairbuf != nullptr;
}

static ColourTiles colour_tiles(const misa_lattice *h, int c) {
    ColourTiles ct;
    ct.nt0 = h->g.nt2[0];
    ct.nt1 = h->g.nt2[1];
    ct.nt2 = h->g.nt2[2];
    ct.colour = c;
    ct.nitems = (ct.nt0 / 2) * (ct.nt1 / 2) * (ct.nt2 / 2);
    ct.nitems_pad = (ct.nitems + 7) / 8 * 8;
    return ct;
}

static Tables<float> half_tables(const misa_lattice *h) {
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    return T;
}

static hipError_t zero_f32(misa_lattice *h, void *a) {
    const int64_t n = h->g.nsites;
    const int64_t b = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_f32, dim3(b > 0 ? b : 1), dim3(256), 0, h->stream, (float *)a, n);
    return hipGetLastError();
}

hipError_t launch_rho_half(misa_lattice *h) {
    const LdsTables &W = h->lds32h;
    hipError_t e = zero_f32(h, h->S.rho);
    if (e != hipSuccess) return e;
    auto kern = W.node_cut ? k_rho_half<true> : k_rho_half<false>;
    for (int c = 0; c < 8; ++c) {
        const ColourTiles ct = colour_tiles(h, c);
        const int grid = std::min(h->persistent_grid, ct.nitems_pad);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(HF_THREADS), 0, h->stream, ct, h->S, h->g, h->half.st, h->half.meta,
                           (const Q4<float> *)W.f, W.inv_hq, W.pcq, W.nwin, (float)h->g.rc2, h->u_cut2,
                           near_args(h, true));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t b = std::min<int64_t>((h->g.nsites + 255) / 256, 8192);
    hipLaunchKernelGGL(k_embed_half, dim3(b > 0 ? b : 1), dim3(256), 0, h->stream, h->S, h->g, half_tables(h),
                       &h->sc.cnt->range_viol);
    return hipGetLastError();
}

static HalfNets half_nets(const misa_lattice *h) {
    HalfNets N;
    N.f = h->mlp.net[0];
    N.phi = h->mlp.net[1];
    N.emb = h->mlp.net[2];
    N.w2f = h->mlp.w2b[0];
    N.w2p = h->mlp.w2b[1];
    N.w2e = h->mlp.w2b[2];
    return N;
}

hipError_t launch_rho_half_mlp(misa_lattice *h) {
    hipError_t e = zero_f32(h, h->S.rho);
    if (e != hipSuccess) return e;
    const HalfNets N = half_nets(h);
    for (int c = 0; c < 8; ++c) {
        const ColourTiles ct = colour_tiles(h, c);
        const int grid = std::min(h->persistent_grid, ct.nitems_pad);
        hipLaunchKernelGGL(k_rho_half_mlp, dim3(grid), dim3(HFM_THREADS), 0, h->stream, ct, h->S, h->g, h->half.st,
                           h->half.meta, N, half_tables(h), (float)h->g.rc2, h->u_cut2, h->pairbuf,
                           near_args(h, true));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t b = std::min<int64_t>((h->g.nsites + 255) / 256, 8192);
    hipLaunchKernelGGL(k_embed_half_mlp, dim3(b > 0 ? b : 1), dim3(256), 0, h->stream, h->S, h->g, N,
                       half_tables(h), &h->sc.cnt->range_viol);
    return hipGetLastError();
}

hipError_t launch_force_half_mlp(misa_lattice *h, bool energy) {
    hipError_t e;
    for (void *a : {h->S.fx, h->S.fy, h->S.fz})
        if ((e = zero_f32(h, a)) != hipSuccess) return e;
    const HalfNets N = half_nets(h);
    auto kern = energy ? k_force_half_mlp<true> : k_force_half_mlp<false>;
    for (int c = 0; c < 8; ++c) {
        const ColourTiles ct = colour_tiles(h, c);
        const int grid = std::min(h->persistent_grid, ct.nitems_pad);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(HFM_THREADS), 0, h->stream, ct, h->S, h->g, h->half.st,
                           h->half.meta, N, half_tables(h), (float)h->g.rc2, h->u_cut2, h->sc.part, h->pairbuf,
                           near_args(h, true));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_force_half(misa_lattice *h, bool energy) {
    const LdsTables &W = h->lds32h;
    hipError_t e;
    for (void *a : {h->S.fx, h->S.fy, h->S.fz})
        if ((e = zero_f32(h, a)) != hipSuccess) return e;
    auto kern = energy ? (W.node_cut ? k_force_half<true, true> : k_force_half<true, false>)
                       : (W.node_cut ? k_force_half<false, true> : k_force_half<false, false>);
    for (int c = 0; c < 8; ++c) {
        const ColourTiles ct = colour_tiles(h, c);
        const int grid = std::min(h->persistent_grid, ct.nitems_pad);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(HF_THREADS), 0, h->stream, ct, h->S, h->g, h->half.st, h->half.meta, W.force,
                           W.inv_hq, W.pcq, W.nwin, half_tables(h), (float)h->g.rc2, h->u_cut2, h->sc.part,
                           near_args(h, true));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace misa
